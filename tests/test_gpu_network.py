"""GPU parity of the learned correction (BF16 MFMA kernels) against the oracle.

The oracle rounds to bfloat16 at the same places as the kernels (inputs,
weights, stored activations and gradients) and computes the rest in FP64, so
the two differ by FP32 accumulation order and by the occasional bf16 rounding
flip that this causes: forward outputs and gradients must agree to 1e-2 in
relative norm (stated per test), far below the size of any indexing or
layout mistake (which gives O(1) errors).
"""
import sys

import numpy as np
import pytest

from workloads import config_c5, random_vector
from oracle import network as onet
from oracle.operator import Problem
from oracle import strip as ostrip

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_05988_amd import sgdg
    sgdg.lib()
    return torch.device("cuda:0")


_cache = {}


def _setup(L=4):
    if L not in _cache:
        from paper_2204_05988_amd import sgdg
        w = config_c5(L=L)
        P = Problem(w)
        ops = sgdg.SparseGridOps(w)
        _cache[L] = (w, P, ops)
    return _cache[L]


def _grid_tensors(w, P, flat, R):
    """[points][R] concatenated -> per-grid tensors [mx, mx, mv, mv, R]."""
    out, off = [], 0
    for lx, lv in P.upper:
        mx, mv = onet.grid_dims(w, lx, lv)
        n = mx * mx * mv * mv
        out.append(flat[off:off + n].reshape(mx, mx, mv, mv, R))
        off += n
    return out


def _relnorm(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_net_forward_parity(dev):
    from paper_2204_05988_amd import sgdg
    w, P, ops = _setup()
    net = sgdg.LearnedPreconditioner(ops, seed=3)
    theta, _ = net.get_params()
    G, R = net.n_grids, P.R
    thetas = theta.astype(np.float64).reshape(G, -1)
    x = random_vector(P.ndof, 12)[0].astype(np.float32)
    _say(f"network forward parity c5 L=4: {G} grids, {P.ndof} points")
    xt = torch.tensor(x, device=dev)
    yt = torch.empty_like(xt)
    net.forward(xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy().astype(np.float64)
    worst = 0.0
    for g, (xg, yg) in enumerate(zip(_grid_tensors(w, P, x.astype(np.float64), R), _grid_tensors(w, P, y, R))):
        ref = onet.forward(thetas[g], xg, w.x.periodic, w.v.periodic, bf16_path=True)[..., :R]
        e = _relnorm(yg, ref)
        worst = max(worst, e)
        assert e <= 1e-2, (g, e)
    _say(f"  worst per-grid relative error {worst:.2e}")
    net.close()


def test_net_backward_parity(dev):
    from paper_2204_05988_amd import sgdg
    w, P, ops = _setup()
    net = sgdg.LearnedPreconditioner(ops, seed=4)
    theta, _ = net.get_params()
    G, R = net.n_grids, P.R
    thetas = theta.astype(np.float64).reshape(G, -1)
    x = random_vector(P.ndof, 13)[0].astype(np.float32)
    dy = random_vector(P.ndof, 14)[0].astype(np.float32)
    _say("network backward parity c5 L=4")
    grad = torch.zeros(net.n_params, dtype=torch.float32, device=dev)
    net.backward(torch.tensor(x, device=dev), torch.tensor(dy, device=dev), grad)
    torch.cuda.synchronize()
    gg = grad.cpu().numpy().astype(np.float64).reshape(G, onet.NCONV, onet.CONV_PARAMS)
    xs = _grid_tensors(w, P, x.astype(np.float64), R)
    dys = _grid_tensors(w, P, dy.astype(np.float64), R)
    worst = 0.0
    for g in range(G):
        dyp = np.zeros(dys[g].shape[:4] + (onet.C,))
        dyp[..., :R] = onet.bf16(dys[g])
        ref, _ = onet.backward(thetas[g], xs[g], dyp, w.x.periodic, w.v.periodic, bf16_path=True)
        ref = ref.reshape(onet.NCONV, onet.CONV_PARAMS)
        for c in range(onet.NCONV):
            e = _relnorm(gg[g, c], ref[c])
            worst = max(worst, e)
            assert e <= 1e-2, (g, c, e)
    _say(f"  worst per-convolution relative gradient error {worst:.2e}")
    net.close()


def test_identity_network_apply(dev):
    """z = s * rms(r) * N(r / rms(r)) with a hand-set identity network equals s * r up to bf16 rounding."""
    from paper_2204_05988_amd import sgdg
    w, P, ops = _setup()
    net = sgdg.LearnedPreconditioner(ops, seed=0)
    G = net.n_grids
    theta = np.zeros(onet.NCONV * onet.CONV_PARAMS)
    convs = [[np.zeros((9, onet.C, onet.C)), np.zeros(onet.C)] for _ in range(onet.NCONV)]
    convs[0][0][4, 0, 0], convs[0][0][4, 1, 0] = 1.0, -1.0
    for c in range(1, 7):
        convs[c][0][4, 0, 0] = convs[c][0][4, 1, 1] = 1.0
    convs[7][0][4, 0, 0], convs[7][0][4, 0, 1] = 1.0, -1.0
    for c in range(onet.NCONV):
        theta[c * onet.CONV_PARAMS:(c + 1) * onet.CONV_PARAMS] = np.concatenate([convs[c][0].ravel(), convs[c][1]])
    scales = np.linspace(0.5, 2.0, G)
    net.set_params(np.tile(theta, G), scales)
    r = random_vector(P.ndof, 15)[0]
    zt = torch.empty(P.ndof, dtype=torch.float64, device=dev)
    _say("identity network through sgdg_net_apply")
    net.apply(torch.tensor(r, device=dev), zt)
    torch.cuda.synchronize()
    ref = np.concatenate([s * b.ravel() for s, b in zip(scales, P.split(r))])
    err = np.abs(zt.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say(f"  max relative error {err:.2e} (bf16 input rounding bound 2^-8)")
    assert err <= 2.0 ** -8
    # random network: apply == oracle apply_learned on the bf16 path
    net.set_params(np.tile(onet_random_theta(), G), scales)
    th, _ = net.get_params()
    net.apply(torch.tensor(r, device=dev), zt)
    torch.cuda.synchronize()
    ref = onet.apply_learned(P, list(th.astype(np.float64).reshape(G, -1)), scales, r, bf16_path=True)
    e = _relnorm(zt.cpu().numpy(), ref)
    _say(f"  random network: relative error vs oracle {e:.2e}")
    assert e <= 1e-2
    net.close()


def onet_random_theta(seed=21):
    rng = np.random.default_rng(seed)
    th = rng.standard_normal(onet.NCONV * onet.CONV_PARAMS) * 0.3 / np.sqrt(9 * onet.C)
    return th


def test_first_adam_step_moves_by_lr(dev):
    from paper_2204_05988_amd import sgdg
    w, P, ops = _setup()
    net = sgdg.LearnedPreconditioner(ops, seed=5)
    r = torch.tensor(random_vector(P.ndof, 16)[0], device=dev)
    z = torch.tensor(random_vector(P.ndof, 17)[0], device=dev)
    net.add_pairs(r, z)
    th0, _ = net.get_params()
    _say("one Adam step")
    net.train(steps=1, batch=1, lr=1e-3, mix=False)
    th1, sc = net.get_params()
    d = np.abs(th1.astype(np.float64) - th0)
    moved = d[d > 0]
    _say(f"  {moved.size} of {d.size} parameters moved; max step {d.max():.3e}")
    assert d.max() <= 1e-3 * (1 + 1e-3)
    # every weight that reaches the output through the first R channels moves by lr (|m/sqrt(v)| = 1)
    assert moved.size > 0.5 * d.size
    assert np.median(moved) >= 0.99e-3
    assert np.all(sc > 0)
    net.close()


def test_learned_preconditioner_trains_and_solves(dev):
    """Pairs recorded from CT-preconditioned solves of strips 1-6 train the
    networks; the learned preconditioner (with CT fallback) then solves strip 7
    to 1e-8, and its gain over CT is reported."""
    from paper_2204_05988_amd import sgdg
    w, P, ops = _setup()
    net = sgdg.LearnedPreconditioner(ops, seed=6)
    net.record(256)
    u = torch.tensor(ostrip.initial_coefficients(P), device=dev)
    prev = 1
    opts = sgdg.default_solve_opts(rtol=1e-8, maxit=200)
    for j in range(1, 7):
        b = ops.rhs(u, prev)
        u, st = ops.solve_strip(b, torch.zeros_like(b), opts)
        prev = P.R
    net.record(0)
    npairs = net.pair_count()
    _say(f"recorded {npairs} (r, P_CT r) pairs from strips 1-6")
    assert npairs >= 8
    ts = net.train(steps=400, batch=8, lr=1e-3, seed=1)
    _say(f"  training: loss {ts.loss_first:.3e} -> {ts.loss_last:.3e} in {ts.seconds:.2f}s")
    assert ts.loss_last < 0.5 * ts.loss_first
    b = ops.rhs(u, prev)
    x_ct, st_ct = ops.solve_strip(b, torch.zeros_like(b), opts)
    lopts = sgdg.default_solve_opts(rtol=1e-8, maxit=300, pc=sgdg.default_precond_opts(net=net))
    x_l, st_l = ops.solve_strip(b, torch.zeros_like(b), lopts)
    bn = b.cpu().numpy()
    res = np.linalg.norm(bn - P.apply(x_l.cpu().numpy())) / np.linalg.norm(bn)
    _say(f"  strip 7: CT {st_ct.outer_iters} iterations {st_ct.seconds:.3f}s; learned {st_l.outer_iters} iterations "
         f"{st_l.seconds:.3f}s (fallback {st_l.fallback_used}, {st_l.pc_applications} applications); "
         f"oracle residual {res:.2e}")
    assert res <= 1.5e-8
    # what training gains: five FGMRES iterations with the learned map alone (no
    # fallback) against the same networks before training (the same seed's initial
    # weights, output scales 1)
    fresh = sgdg.LearnedPreconditioner(ops, seed=6)
    probe = sgdg.default_solve_opts(rtol=1e-14, maxit=5, restart=5,
                                    pc=sgdg.default_precond_opts(net=net, fallback_iters=1000))
    _, st_t = ops.solve_strip(b, torch.zeros_like(b), probe, raise_on_noconv=False)
    probe.pc.net = fresh.h
    _, st_f = ops.solve_strip(b, torch.zeros_like(b), probe, raise_on_noconv=False)
    _say(f"  five learned iterations: trained residual {st_t.rel_residual:.3e}, untrained {st_f.rel_residual:.3e} "
         f"(gain {st_f.rel_residual / st_t.rel_residual:.2f}x); against CT: {st_l.seconds / st_ct.seconds:.2f}x the CT time")
    assert st_t.rel_residual < st_f.rel_residual
    fresh.close()
    net.close()


def test_net_parity_at_benchmark_size(dev):
    """c5 at L = 7, the size the benchmark trains and runs at: forward outputs and
    weight gradients of the largest x-grid (7, 0) and the largest v-grid (0, 7)
    against the oracle (1e-2 relative norm, as above).  The networks of different
    grids share nothing, so each grid's slice of the full launch is checked alone."""
    from paper_2204_05988_amd import sgdg
    w, P, ops = _setup(7)
    net = sgdg.LearnedPreconditioner(ops, seed=8)
    theta, _ = net.get_params()
    G, R = net.n_grids, P.R
    thetas = theta.astype(np.float64).reshape(G, -1)
    x = random_vector(P.ndof, 18)[0].astype(np.float32)
    dy = random_vector(P.ndof, 19)[0].astype(np.float32)
    _say(f"network parity c5 L=7: {G} grids, {P.ndof} points")
    xt = torch.tensor(x, device=dev)
    yt = torch.empty_like(xt)
    net.forward(xt, yt)
    grad = torch.zeros(net.n_params, dtype=torch.float32, device=dev)
    net.backward(xt, torch.tensor(dy, device=dev), grad)
    torch.cuda.synchronize()
    y = yt.cpu().numpy().astype(np.float64)
    gg = grad.cpu().numpy().astype(np.float64).reshape(G, onet.NCONV, onet.CONV_PARAMS)
    xs = _grid_tensors(w, P, x.astype(np.float64), R)
    ys = _grid_tensors(w, P, y, R)
    dys = _grid_tensors(w, P, dy.astype(np.float64), R)
    picks = [P.upper.index((w.L, w.lmin)), P.upper.index((w.lmin, w.L))]
    for g in picks:
        ref = onet.forward(thetas[g], xs[g], w.x.periodic, w.v.periodic, bf16_path=True)[..., :R]
        e = _relnorm(ys[g], ref)
        dyp = np.zeros(dys[g].shape[:4] + (onet.C,))
        dyp[..., :R] = onet.bf16(dys[g])
        gref, _ = onet.backward(thetas[g], xs[g], dyp, w.x.periodic, w.v.periodic, bf16_path=True)
        gref = gref.reshape(onet.NCONV, onet.CONV_PARAMS)
        eg = max(_relnorm(gg[g, c], gref[c]) for c in range(onet.NCONV))
        _say(f"  grid {P.upper[g]}: forward {e:.2e}, worst convolution gradient {eg:.2e}")
        assert e <= 1e-2
        assert eg <= 1e-2
    net.close()


def test_batched_learned_mixed_solve(dev):
    """Two 4D Vlasov-type problems (different seeds, so different fields E) in one
    batch, each with its own network (trained briefly on pairs recorded from its
    own CT solves): the batched learned + mixed-precision solve reaches 1e-8 under
    each problem's oracle operator, with and without the CT fallback taking over;
    a batch solve with a learned preconditioner but no networks is refused."""
    from paper_2204_05988_amd import sgdg
    probs = []
    for seed in (0, 1):
        w = config_c5(seed=seed, L=4)
        P = Problem(w)
        ops = sgdg.SparseGridOps(w)
        net = sgdg.LearnedPreconditioner(ops, seed=10 + seed)
        net.record(64)
        u = torch.tensor(ostrip.initial_coefficients(P), device=dev)
        for j in range(1, 4):
            b = ops.rhs(u, 1)
            u, _ = ops.solve_strip(b, torch.zeros_like(b), sgdg.default_solve_opts(rtol=1e-8))
        net.record(0)
        ts = net.train(steps=150, batch=8, lr=1e-3, seed=2)
        _say(f"problem seed {seed}: {net.pair_count()} pairs, loss {ts.loss_first:.3e} -> {ts.loss_last:.3e}")
        probs.append((w, P, ops, net, ops.rhs(u, 1)))
    batch = sgdg.SparseGridBatch([p[2] for p in probs])
    off = batch.offsets
    bt = torch.cat([p[4] for p in probs])
    bn = bt.cpu().numpy()
    opts = sgdg.default_solve_opts(rtol=1e-8, maxit=300, mixed=True,
                                   pc=sgdg.default_precond_opts(net=probs[0][3]))
    with pytest.raises(sgdg.SgdgError):
        batch.solve(bt, torch.zeros_like(bt), opts)
    batch.set_networks([p[3] for p in probs])
    for drop, label in ((10.0, "default fallback rule"), (1e30, "fallback at the first check")):
        opts.pc.fallback_drop = drop
        x, st = batch.solve(bt, torch.zeros_like(bt), opts)
        xs = x.cpu().numpy()
        _say(f"  batched learned+mixed ({label}): {st.outer_iters} iterations, {st.refinement_steps} refinements, "
             f"fallback {st.fallback_used}, {st.pc_applications} applications, {st.seconds:.3f}s")
        for k, (w, P, ops, net, b) in enumerate(probs):
            res = np.linalg.norm(bn[off[k]:off[k + 1]] - P.apply(xs[off[k]:off[k + 1]])) / \
                np.linalg.norm(bn[off[k]:off[k + 1]])
            _say(f"    problem {k}: oracle residual {res:.2e}")
            assert res <= 1e-8 * (1 + 1e-6)
    assert st.fallback_used == 1
    batch.close()
    for p in probs:
        p[3].close()
