"""Benchmark: sparse-grid SD-DG operator application on one MI355X.

One step = one application of the full strip operator A^(delta) (all blocks
A_{l,l'} of every component-grid pair: per-grid Kronecker sweeps, cross-grid
level scans with the embedding matrices, term accumulation) to a batch of
synthetic input vectors already resident in HBM.  Workload: the 4D phase-space
problem (d=2, r=1, sparse-grid level 7, 620 892 space-time DOFs per vector).

Prints one JSON line (rank 0).  Also reports, beside the headline number:
  * strip_solve: the first strip of that problem solved to 1e-8 in FP64 and in
    mixed precision (FP32 inner, FP64 refinement);
  * learned: the 4D Vlasov-type step (x periodic, frozen random E(x), L=7,
    r=0): (r, P_CT r) pairs recorded from CT-preconditioned solves of strips
    1-8, the per-grid networks trained on them, then strips 9-10 solved to 1e-8
    with CT, with the learned preconditioner, and learned + mixed precision,
    and again with inexact CT grid solves (10 GMRES iterations) as CT and as
    the learned preconditioner's fallback, in FP64 and in mixed precision;
    its "network" entry is the forward rate of the trained network against
    the HBM roofline, with its matrix-core utilisation (--network-only: that
    rate alone, freshly initialised);
  * batched: independent 4D problems with levels drawn from {5,6,7}, applied
    and solved in lockstep (FP32 applies inside FP64 refinement) against the
    same problems solved one at a time in plain FP64;
  * apply_6d: the 6D phase-space problem (d=3, L=6) applied in FP64 and FP32;
  * apply_2d: the 2D phase-space problem (d=1, L=6) applied to a batch, and
    its 8-strip march with CT-preconditioned FGMRES to 1e-10;
  * cpu_baseline: the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense bf16 matrix-core peak
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 157.3  # non-packed FP32: twice the FP64 lane rate


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--level", type=int, default=7)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--batched", type=int, default=64, help="problems of the batched leg (0 = skip)")
    ap.add_argument("--c3-level", type=int, default=6, help="level of the 6D apply leg (0 = skip)")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--network-only", action="store_true",
                    help="learned leg reduced to the network's forward rate (freshly initialised weights)")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D phase-space (d=1) leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed loop, copy a 512 MiB buffer once (calibrates HBM byte counters)")
    return ap.parse_args()


def kernel_work(ops, B, R, elem_bytes):
    """Algorithmic flops and HBM bytes per launch of each operator kernel.

    Per point of upper grid i (of n) and per vector, with nt Kronecker terms,
    nvg / nxg distinct v- / x-factors, S-point stencils (S = 3, 7, 15 for
    d = 1, 2, 3) and R time slices:
      k_vstage  W^m = sum_{k in m} Tm_k [V_k u + E^x Pt^{j(k)}]:
                flops nt R 2S + nt 2R^2 (+ nt R 4 if i > 0);
                bytes u (R) + W (nxg R) [+ Pt (nt R / 2^d) if i > 0]
      k_ustage  sum_k Tm_k (V_k E^v) Qt^{m(k)}, i < n-1 (zero fill otherwise); d <= 2
                with the prolongated stencils V_k E^v (3^d coarse nodes per fine node):
                flops nt (R 2 3^d + 2R^2); d = 3 prolonging Qt on the fly:
                flops nxg S R 4 + nt (R 2S + 2R^2); bytes Qt (nxg R / 2^d) + y (R)
      k_xstage  y += sum_m X_m W^m:  flops nxg R 2S; bytes W (nxg R) + y (2R)
                (the same counts for k_xtile, its LDS-tiled form: halo re-reads are not algorithmic)
      k_fused   the whole block row from LDS-staged boxes:
                flops nvg R (2S + 4) + nt R (2S + 2R) [+ nxg R 4 + nt R (2S + 2R) if i < n-1];
                bytes u (R) + y (R) + Pt, Qt (nvg R / 2^d, nxg R / 2^d)
    The partner scan arrays live on the lower diagonal, 2^d times smaller.
    Face masses vanish off their face: in the split passes the X-group counts
    and the terms above are the per-x-node averages of where each group can
    contribute (sgdg_op_support): W^m staged where a nonzero row's stencil
    reads it (v-stage work, x-stage W reads), rows with a nonzero (x-stage
    flops), and where Qt^m can be nonzero (upper-partner pass).
    """
    info = ops.op_info()
    nt, nvg, nxg = info["nterms"], info["nvg"], info["nxg"]
    d = ops.w.d
    S = {1: 3, 2: 7, 3: 15}[d]
    n = len(ops.upper)
    work = {k: [0.0, 0.0] for k in ("vstage", "ustage", "xstage", "fused")}
    for gi, (lx, _, nx, nv) in enumerate(ops.upper):
        pts = nx * nv * B
        hp, hq = gi > 0, gi + 1 < n
        sup = ops.op_support(lx)
        rt, rg = sup["read_terms"] / sup["nodes"], sup["read_groups"] / sup["nodes"]
        wg = sup["row_groups"] / sup["nodes"]
        qg, qtt = sup["qt_groups"] / sup["nodes"], sup["qt_terms"] / sup["nodes"]

        def add(k, fl, by):
            work[k][0] += pts * fl
            work[k][1] += pts * by * elem_bytes
        add("vstage", rt * R * 2 * S + rt * 2 * R * R + (rt * R * 4 if hp else 0),
            R + rg * R + (rt * R / 2 ** d if hp else 0))
        uf = qtt * (R * 2 * 3 ** d + 2 * R * R) if d <= 2 else qg * S * R * 4 + qtt * (R * 2 * S + 2 * R * R)
        add("ustage", uf if hq else 0,
            (qg * R / 2 ** d if hq else 0) + R)
        add("xstage", wg * R * 2 * S, rg * R + 2 * R)
        add("fused", nvg * R * (2 * S + 4) + nt * R * (2 * S + 2 * R) + ((nxg * R * 4 + nt * R * (2 * S + 2 * R)) if hq else 0),
            2 * R + (nvg * R / 2 ** d if hp else 0) + (nxg * R / 2 ** d if hq else 0))
    return work


def recorded_traffic(kernel, workload_tag):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary of this workload, or None if there is none or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"apply_{workload_tag}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    src = {"k_vstage": "split.hip", "k_ustage": "split.hip", "k_xstage": "split.hip", "k_xtile": "split.hip",
           "k_scan2": "fused.hip", "k_fused": "fused.hip"}.get(kernel)
    if src is None:
        return None
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2204_05988_amd", "csrc", src), "rb").read()).hexdigest()[:16]
    text = open(path).read()
    if f"{src} sha256/16 {sha}" not in text:
        return None
    for line in text.splitlines():
        f = line.split()
        if f and f[0] == kernel:
            return float(f[4])
    return None


def roofline(fl, by, ms, valu_peak):
    t_hbm = by / (HBM_PEAK_GBS * 1e9)
    t_alu = fl / (valu_peak * 1e12)
    if t_alu > t_hbm:
        ach = fl / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(ach, 3), "peak": valu_peak, "unit": "TFLOP/s",
                "frac": round(ach / valu_peak, 4)}
    ach = by / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4)}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; execution across several GPUs is not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import config_c2, random_vector

    dev = torch.device("cuda:0")
    w = config_c2(L=a.level)
    ops = sgdg.SparseGridOps(w)
    R = w.r + 1
    B = a.batch
    dt = torch.float64 if a.dtype == "f64" else torch.float32
    u = torch.tensor(random_vector(ops.ndof, 0, batch=B), device=dev, dtype=dt)
    y = torch.empty_like(u)
    stream = torch.cuda.current_stream()
    tuned = None if a.no_tune else ops.tune(a.dtype, batch=B, reps=3)
    if tuned is not None:
        _log(f"launch configuration: {tuned}")
    for _ in range(a.warmup):
        ops.apply(u, y, batch=B)
    torch.cuda.synchronize()
    ops.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(a.steps):
        ops.apply(u, y, batch=B)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    slots = {"scan": 0, "fused": 1, "vstage": 3, "ustage": 4, "xstage": 5}
    prof = {name: ops.profile_read(slot) for name, slot in slots.items()}
    prof = {k: v for k, v in prof.items() if v[1] > 0}
    ops.profile(False)
    ms_step = ms / a.steps
    value = B * ops.ndof / (ms_step * 1e-3)
    valu_peak = FP64_VALU_PEAK_TFLOPS if a.dtype == "f64" else FP32_VALU_PEAK_TFLOPS
    work = kernel_work(ops, B, R, 8 if a.dtype == "f64" else 4)
    per_kernel = {}
    for k, (tot, cnt) in prof.items():
        if k in work and cnt > 0:
            kms = tot / cnt
            per_kernel[k] = dict(roofline(work[k][0], work[k][1], kms, valu_peak), kernel_ms=round(kms, 4),
                                 flops=work[k][0], bytes=work[k][1])
    # the x-stage slot times the tiled kernel when the tuner picked it
    kname = {k: "k_" + k for k in per_kernel}
    if tuned is not None and tuned.get("variant") == "split_tiled" and "xstage" in kname:
        kname["xstage"] = "k_xtile"
    dom = max(per_kernel, key=lambda k: per_kernel[k]["kernel_ms"])
    roof = dict(per_kernel[dom])
    roof["kernel"] = kname[dom]
    tag = f"c2_L{a.level}_B{B}_{a.dtype}"
    roof["traffic"] = recorded_traffic(kname[dom], tag)
    out = {
        "metric": "DOF-applies/s", "value": value, "unit": "DOF-applies/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": a.dtype, "data": "synthetic",
        "config": {"workload": f"4D phase space d=2, r=1, sparse grid L={a.level} (c2), full SD-DG operator",
                   "dofs_per_vector": ops.ndof, "batch": B, "grids": len(ops.upper)},
        "kernel_ms_per_step": {k: round(v[0] / a.steps, 4) for k, v in prof.items()},
        "launch_config": tuned,
        "dominant_kernel": kname[dom],
        "kernel_names": kname,
        "roofline": roof,
        "kernels": per_kernel,
        "wall_s": round(wall, 3),
    }
    _log(f"apply: {value:.3e} DOF-applies/s")
    if a.calib_copy:
        src = torch.empty(64 * 2 ** 20, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        _log("calibration copy: 512 MiB read + 512 MiB written")
    if not a.no_solve:
        out["strip_solve"] = solve_times(ops, w, dev)
        _log(f"strip solves: {out['strip_solve']}")
    if a.network_only:
        out["network"] = network_leg(dev)
    elif not a.no_learned:
        out["learned"] = learned_leg(dev, a.train_steps)
    if a.batched > 0:
        out["batched"] = batched_leg(dev, a.batched)
    if a.c3_level > 0:
        out["apply_6d"] = apply_6d_leg(dev, a.c3_level)
    if not a.no_2d:
        out["apply_2d"] = apply_2d_leg(dev)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, value)
    print(json.dumps(out), flush=True)


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def solve_times(ops, w, dev):
    """One strip (the first) of the c2 problem to 1e-8: FP64 and mixed precision."""
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import gauss_legendre_times, sample_on_grids, lattice_coords
    R = w.r + 1
    # U_0 = sparse-grid interpolant of u0 (combination of nodal values), on the device
    nodal0 = np.concatenate([sample_on_grids(w, _grids(ops.upper), w.u0), sample_on_grids(w, _grids(ops.lower), w.u0)])
    u0 = torch.empty(ops.npts_up, dtype=torch.float64, device=dev)
    ops.combine(torch.tensor(nodal0, device=dev), u0, 1)
    nq = w.r + 2
    tq, _ = gauss_legendre_times(0.0, w.dt, nq)

    def nodal(fn):
        return torch.tensor(np.stack([np.concatenate([sample_on_grids(w, _grids(ops.upper), fn, t),
                                                      sample_on_grids(w, _grids(ops.lower), fn, t)]) for t in tq]),
                            device=dev)

    b = ops.rhs(u0, 1, nodal(w.f), nodal(w.g))
    res = {}
    # grid problems to 1e-8 (at most 200 GMRES iterations), and inexact (10 iterations each)
    for name, mixed, cap in (("fp64", False, 200), ("mixed_fp32", True, 200),
                             ("fp64_inexact_ct", False, 10), ("mixed_fp32_inexact_ct", True, 10)):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        opts = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=mixed,
                                       pc=sgdg.default_precond_opts(inner_maxit=cap))
        x, st = ops.solve_strip(b, x, opts, raise_on_noconv=False)
        torch.cuda.synchronize()
        res[name] = {"seconds": round(time.perf_counter() - t0, 4), "outer_iters": st.outer_iters,
                     "inner_iters": st.inner_iters_total, "rel_residual": st.rel_residual,
                     "refinements": st.refinement_steps}
    return res


def _interp_u0(ops, w, dev):
    """Spanning coefficients of the sparse-grid interpolant of u0 (combination on the device)."""
    import torch
    from workloads import sample_on_grids
    nodal0 = np.concatenate([sample_on_grids(w, _grids(ops.upper), w.u0), sample_on_grids(w, _grids(ops.lower), w.u0)])
    u0 = torch.empty(ops.npts_up, dtype=torch.float64, device=dev)
    ops.combine(torch.tensor(nodal0, device=dev), u0, 1)
    return u0


def _timed_solve(ops, b, opts):
    import torch
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = ops.solve_strip(b, x, opts, raise_on_noconv=False)
    torch.cuda.synchronize()
    return x, {"seconds": round(time.perf_counter() - t0, 4), "outer_iters": st.outer_iters,
               "inner_iters": st.inner_iters_total, "rel_residual": st.rel_residual,
               "pc_applications": st.pc_applications, "fallback": st.fallback_used}


def learned_leg(dev, train_steps, L=7, record_strips=8, test_strips=2):
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import config_c5
    w = config_c5(L=L)
    t0 = time.perf_counter()
    ops = sgdg.SparseGridOps(w)
    setup = time.perf_counter() - t0
    net = sgdg.LearnedPreconditioner(ops, seed=0)
    u = _interp_u0(ops, w, dev)
    prev = 1
    ct = sgdg.default_solve_opts(rtol=1e-8, maxit=400)
    net.record(4096)
    rec_time = 0.0
    for j in range(1, record_strips + 1):
        b = ops.rhs(u, prev)
        u, st = _timed_solve(ops, b, ct)
        rec_time += st["seconds"]
        prev = 1
        _log(f"learned leg: CT strip {j} {st}")
    net.record(0)
    ts = net.train(train_steps, batch=8, lr=1e-3, seed=1)
    _log(f"learned leg: trained {ts.steps} steps in {ts.seconds:.2f}s, loss {ts.loss_first:.3e} -> {ts.loss_last:.3e}")
    out = {"workload": f"4D Vlasov-type step, x periodic, E(x) 16 modes, L={L}, r=0 (c5)", "dofs": ops.ndof,
           "setup_s": round(setup, 3), "pairs": net.pair_count(), "record_strips": record_strips,
           "record_solve_s": round(rec_time, 3),
           "train": {"steps": ts.steps, "batch": 8, "seconds": round(ts.seconds, 3),
                     "loss_first": ts.loss_first, "loss_last": ts.loss_last}, "strips": []}
    out["network"] = network_rate(net, ops, dev)
    _log(f"learned leg: network {out['network']}")
    learned = sgdg.default_solve_opts(rtol=1e-8, maxit=400, pc=sgdg.default_precond_opts(net=net))
    learned_mixed = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True, pc=sgdg.default_precond_opts(net=net))
    # inexact grid problems (10 GMRES iterations each): the combination technique
    # alone, and as the learned preconditioner's fallback
    ct_inexact = sgdg.default_solve_opts(rtol=1e-8, maxit=400, pc=sgdg.default_precond_opts(inner_maxit=10))
    learned_inexact = sgdg.default_solve_opts(rtol=1e-8, maxit=400,
                                              pc=sgdg.default_precond_opts(net=net, inner_maxit=10))
    learned_inexact_mixed = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True,
                                                    pc=sgdg.default_precond_opts(net=net, inner_maxit=10))
    for j in range(record_strips + 1, record_strips + test_strips + 1):
        b = ops.rhs(u, prev)
        row = {"strip": j}
        x, row["ct_fp64"] = _timed_solve(ops, b, ct)
        _, row["learned_fp64"] = _timed_solve(ops, b, learned)
        _, row["learned_mixed"] = _timed_solve(ops, b, learned_mixed)
        _, row["ct_inexact_fp64"] = _timed_solve(ops, b, ct_inexact)
        _, row["learned_inexact_fallback_fp64"] = _timed_solve(ops, b, learned_inexact)
        _, row["learned_inexact_fallback_mixed"] = _timed_solve(ops, b, learned_inexact_mixed)
        t0 = row["ct_fp64"]["seconds"]
        row["gain_vs_ct_fp64"] = {k: round(t0 / row[k]["seconds"], 3)
                                  for k in ("learned_fp64", "learned_mixed", "ct_inexact_fp64",
                                            "learned_inexact_fallback_fp64", "learned_inexact_fallback_mixed")}
        out["strips"].append(row)
        _log(f"learned leg: {row}")
        u = x
    net.close()
    ops.close()
    return out


def network_leg(dev, L=7):
    from paper_2204_05988_amd import sgdg
    from workloads import config_c5
    ops = sgdg.SparseGridOps(config_c5(L=L))
    net = sgdg.LearnedPreconditioner(ops, seed=0)
    out = dict(network_rate(net, ops, dev), workload=f"c5 L={L}, one residual, all grids")
    _log(f"network: {out}")
    net.close()
    ops.close()
    return out


def network_rate(net, ops, dev, reps=20):
    """Forward of the trained network on one residual-sized input (all grids,
    channels-last [points][R] FP32), timed with events on the launching stream.
    MFMA work issued: 8 convolutions x 9 taps x 32 x 32 channels x 2 flops per
    point (the padded input and output channels included)."""
    import torch
    R = ops.R
    x = torch.randn(ops.ndof, dtype=torch.float32, device=dev, generator=torch.Generator(dev).manual_seed(3))
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        net.forward(x, y, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        net.forward(x, y, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    points = ops.ndof // R
    flops = 8 * 9 * 32 * 32 * 2 * points
    # HBM bytes of the 8 convolutions: each reads its bf16 input (64 B per point)
    # once and writes 64 B (the last, FP32, 128 B); 4.0 GFLOP per 28 MB is
    # 144 flop/B, below the bf16 ridge point (2500 / 8 = 312 flop/B), so the
    # convolutions are HBM-bound and the matrix-core fraction is the utilisation
    nbytes = points * (7 * 128 + 64 + 128)
    tf = flops / (ms * 1e-3) / 1e12
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"points": points, "forward_ms": round(ms, 4), "mfma_flops": flops, "bytes": nbytes,
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "mfma": {"achieved": round(tf, 2), "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "utilisation": round(tf / BF16_MFMA_PEAK_TFLOPS, 5)}}


def apply_6d_leg(dev, L, steps=5):
    """Operator-apply throughput of the 6D phase-space problem (d=3, r=0), one vector, FP64 and FP32."""
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import config_c3, random_vector
    w = config_c3(L=L)
    t0 = time.perf_counter()
    ops = sgdg.SparseGridOps(w)
    setup = time.perf_counter() - t0
    _log(f"6d leg: L={L}, {ops.ndof} DOFs, assembled in {setup:.1f}s")
    out = {"workload": f"6D phase space d=3, r=0, sparse grid L={L} (c3), full SD-DG operator", "dofs": ops.ndof,
           "grids": len(ops.upper), "setup_s": round(setup, 2)}
    u64 = torch.tensor(random_vector(ops.ndof, 0)[0], device=dev)
    for name, u in (("f64", u64), ("f32", u64.float())):
        tuned = ops.tune(name, batch=1, reps=2)
        y = torch.empty_like(u)
        ops.apply(u, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ops.apply(u, y)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        out[name] = {"ms": round(el * 1e3, 3), "dof_applies_per_s": ops.ndof / el, "launch_config": tuned}
        _log(f"6d leg: {name} {out[name]}")
    ops.close()
    return out


def apply_2d_leg(dev, batch=64, steps=20):
    """2D phase space (d=1, c1): apply throughput for `batch` vectors in FP64, and the
    plain method's 8-strip march (CT-preconditioned FGMRES to 1e-10 per strip)."""
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import config_c1, gauss_legendre_times, random_vector, sample_on_grids
    w = config_c1()
    ops = sgdg.SparseGridOps(w)
    out = {"workload": f"2D phase space d=1, r={w.r}, sparse grid L={w.L} (c1), full SD-DG operator",
           "dofs": ops.ndof, "grids": len(ops.upper), "batch": batch}
    u = torch.tensor(random_vector(ops.ndof, 0, batch=batch), device=dev)
    y = torch.empty_like(u)
    tuned = ops.tune("f64", batch=batch, reps=3)
    ops.apply(u, y, batch=batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ops.apply(u, y, batch=batch)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    out["apply_f64"] = {"ms": round(el * 1e3, 4), "dof_applies_per_s": batch * ops.ndof / el, "launch_config": tuned}
    # the march: u_0 interpolated, then per strip rhs (jump + inflow data) and solve
    u_prev = _interp_u0(ops, w, dev)
    prev_slices = 1
    nq = w.r + 2
    opts = sgdg.default_solve_opts(rtol=1e-10, maxit=150)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for j in range(1, w.nstrips + 1):
        tq, _ = gauss_legendre_times((j - 1) * w.dt, w.dt, nq)
        g = None
        if w.g is not None:
            g = torch.tensor(np.stack([np.concatenate([sample_on_grids(w, _grids(ops.upper), w.g, t),
                                                       sample_on_grids(w, _grids(ops.lower), w.g, t)]) for t in tq]),
                             device=dev)
        b = ops.rhs(u_prev, prev_slices, None, g)
        x, st = ops.solve_strip(b, torch.zeros_like(b), opts, raise_on_noconv=False)
        iters.append(st.outer_iters)
        u_prev, prev_slices = x, ops.R
    torch.cuda.synchronize()
    out["march"] = {"strips": w.nstrips, "seconds": round(time.perf_counter() - t0, 4), "outer_iters": iters,
                    "last_rel_residual": st.rel_residual, "note": "includes the host sampling of the inflow data"}
    _log(f"2d leg: {out}")
    ops.close()
    return out


def batched_leg(dev, n):
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import config_c4, gauss_legendre_times, sample_on_grids
    members = config_c4(seed=0, n=n)
    t0 = time.perf_counter()
    ops_list = [sgdg.SparseGridOps(w) for w in members]
    setup = time.perf_counter() - t0
    _log(f"batched leg: {n} problems assembled in {setup:.1f}s")
    batch = sgdg.SparseGridBatch(ops_list)
    # strip 1 right-hand sides: u0 = 0, forcing f at the Gauss points of the strip
    bs = []
    for w, ops in zip(members, ops_list):
        tq, _ = gauss_legendre_times(0.0, w.dt, w.r + 2)
        f = torch.tensor(np.stack([np.concatenate([sample_on_grids(w, _grids(ops.upper), w.f, t),
                                                   sample_on_grids(w, _grids(ops.lower), w.f, t)]) for t in tq]),
                         device=dev)
        zero = torch.zeros(ops.npts_up, dtype=torch.float64, device=dev)
        bs.append(ops.rhs(zero, 1, f, None))
    b = torch.cat(bs)
    out = {"workload": f"{n} independent 4D problems, levels {{5,6,7}}, beta=(v,a_i), sigma_i, Fourier forcing (c4)",
           "problems": n, "levels": [w.L for w in members], "dofs_total": batch.ndof, "setup_s": round(setup, 3)}
    # batched apply throughput
    for name, dt in (("apply_f64", torch.float64), ("apply_f32", torch.float32)):
        u = torch.randn(batch.ndof, dtype=dt, device=dev)
        y = torch.empty_like(u)
        for _ in range(3):
            batch.apply(u, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 10
        for _ in range(reps):
            batch.apply(u, y)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        out[name] = {"ms": round(el * 1e3, 3), "dof_applies_per_s": batch.ndof / el}
    # lockstep mixed-precision solve vs one-at-a-time FP64
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = batch.solve(b, x, sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True), raise_on_noconv=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    out["batched_mixed_solve"] = {"seconds": round(tb, 3), "outer_iters": st.outer_iters,
                                  "refinements": st.refinement_steps, "max_rel_residual": st.rel_residual}
    _log(f"batched leg: {out['batched_mixed_solve']}")
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = batch.solve(b, x, sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True,
                                                      pc=sgdg.default_precond_opts(inner_maxit=10)),
                        raise_on_noconv=False)
    torch.cuda.synchronize()
    tbi = time.perf_counter() - t0
    out["batched_mixed_solve_inexact_ct"] = {"seconds": round(tbi, 3), "outer_iters": st.outer_iters,
                                             "refinements": st.refinement_steps, "max_rel_residual": st.rel_residual}
    _log(f"batched leg: {out['batched_mixed_solve_inexact_ct']}")
    seq, worst = 0.0, 0.0
    for ops, bb in zip(ops_list, bs):
        _, r = _timed_solve(ops, bb, sgdg.default_solve_opts(rtol=1e-8, maxit=400))
        seq += r["seconds"]
        worst = max(worst, r["rel_residual"])
    out["sequential_fp64_solve"] = {"seconds": round(seq, 3), "max_rel_residual": worst}
    out["speedup_batched_mixed_vs_sequential_fp64"] = round(seq / tb, 3)
    out["speedup_batched_mixed_inexact_ct_vs_sequential_fp64"] = round(seq / tbi, 3)
    batch.close()
    for o in ops_list:
        o.close()
    return out


def _grids(shapes):
    return [(lx, lv) for lx, lv, _, _ in shapes]


_CPU_P = None   # the oracle problem shared with forked pool workers


def _cpu_rows(idx):
    """Worker: output blocks [A u]_l for the upper grids in idx (the blocks are independent)."""
    P, u = _CPU_P
    blocks = P.split(u)
    out = []
    for i in idx:
        l = P.upper[i]
        y = sum(P.block_apply(P.terms, l, l2, ub) for l2, ub in zip(P.upper, blocks))
        out.append((i, y.ravel()))
    return out


def _cpu_info():
    info = {"cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        info["blas"] = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()]
    except Exception:  # pragma: no cover
        pass
    return info


def cpu_baseline(w, gpu_value, gpu_strips=None):
    """The oracle (factored form, NumPy/SciPy FP64) on the host cores.

    apply: single-vector applies of the headline operator on one core (BLAS
    limited to one thread), and on all cores as a process pool over the output
    grids (each block row [A u]_l = sum_l' A_{l,l'} u_l' is independent);
    strips: FGMRES to 1e-8 with the oracle's combination technique (direct
    grid solves) for the 8-strip 2D march and one strip of the 4D problems at
    L = 5 (the L = 7 strips take minutes on the host)."""
    global _CPU_P
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle.operator import Problem
    from oracle.ct import CTPreconditioner
    from oracle.krylov import fgmres
    from oracle import strip as ostrip
    from workloads import config_c1, config_c2, config_c5, random_vector
    info = _cpu_info()
    ncores = info["affinity"]
    out = {"kind": "oracle", "unit": "DOF-applies/s", "host": info}
    with threadpool_limits(1):
        P = Problem(w)
        u = random_vector(P.ndof, 0)[0]
        t0 = time.perf_counter()
        P.apply(u)   # the first apply also builds the factor caches
        setup = time.perf_counter() - t0
        n = 0
        t0 = time.perf_counter()
        while n < 3 or (time.perf_counter() - t0 < 6.0 and n < 20):
            P.apply(u)
            n += 1
        v1 = n * P.ndof / (time.perf_counter() - t0)
        out["single_core"] = {"value": v1, "cores": 1, "sample": f"{n} single-vector applies after a {setup:.1f}s factor setup"}
        # all cores: fork after the caches exist, one task per output grid, largest first
        _CPU_P = (P, u)
        order = sorted(range(len(P.upper)), key=lambda i: -P.sizes[i])
        workers = max(1, min(ncores, len(order)))
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            pool.map(_cpu_rows, [[i] for i in order])
            k = 0
            t0 = time.perf_counter()
            while k < 3 or (time.perf_counter() - t0 < 6.0 and k < 20):
                pool.map(_cpu_rows, [[i] for i in order], chunksize=1)
                k += 1
            vall = k * P.ndof / (time.perf_counter() - t0)
        _CPU_P = None
        out.update(value=vall, cores=workers,
                   sample=f"{k} single-vector applies of the c2 operator (L={w.L}, {P.ndof} DOFs), {workers} worker "
                          f"processes over the {len(P.upper)} output grids, one BLAS thread each")
        out["gpu_over_cpu"] = gpu_value / vall
        strips = {}
        for name, wk, nst, tol in (("c1_march", config_c1(), 8, 1e-10), ("c2_L5_strip1", config_c2(L=5), 1, 1e-8),
                                   ("c5_L5_strip1", config_c5(L=5), 1, 1e-8)):
            t0 = time.perf_counter()
            Pk = Problem(wk)
            ct = CTPreconditioner(Pk)
            uprev, prev = ostrip.initial_coefficients(Pk), 1
            its = []
            for j in range(1, nst + 1):
                b = ostrip.rhs(Pk, j, uprev, prev)
                x, st = fgmres(Pk.apply, b, ct, tol=tol, restart=50, maxit=300)
                its.append(st["iters"])
                uprev, prev = x, Pk.R
            strips[name] = {"seconds": round(time.perf_counter() - t0, 3), "dofs": Pk.ndof, "strips": nst,
                            "outer_iters": its, "rtol": tol, "cores": 1}
            if gpu_strips and name in gpu_strips:
                strips[name]["gpu_seconds"] = gpu_strips[name]
            _log(f"cpu baseline: {name} {strips[name]}")
        out["strips"] = strips
    return out


if __name__ == "__main__":
    main()
