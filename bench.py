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
    with CT, with the learned preconditioner, and learned + mixed precision;
  * batched: independent 4D problems with levels drawn from {5,6,7}, applied
    and solved in lockstep (FP32 applies inside FP64 refinement) against the
    same problems solved one at a time in plain FP64;
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
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz


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
    ap.add_argument("--train-steps", type=int, default=300)
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed loop, copy a 512 MiB buffer once (calibrates HBM byte counters)")
    return ap.parse_args()


def kernel_roofline(ops, shapes, B, R, elem_bytes):
    """Algorithmic flops and bytes per launch of the fused accumulation kernel (k_fused).

    Per output point of upper grid i and per vector:
      diagonal+lower part: for every V-group j, Z_j = V_j u + E^x Pt_j   (Rin (2 Sv + 4) flops)
                           for every term k, Rin x-stencil sums of Sx entries and an Rout x Rin mix
      upper part (i < n-1): for every X-group m, E^v Qt_m                  (Rin 4 flops)
                           for every term k, Rin v-stencil sums of Sv entries and the mix
    Bytes: u read once (Rin), y written once (Rout), the lower-diagonal scan
    arrays read once per group (they are 2^d times smaller than the grid).
    Box halos are not counted (they are implementation overhead, not algorithm).
    """
    info = ops.op_info()
    nt, nvg, nxg, Sx, Sv = info["nterms"], info["nvg"], info["nxg"], info["Sx"], info["Sv"]
    d = ops.w.d
    flops = 0.0
    bytes_ = 0.0
    n = len(shapes)
    for gi, (_, _, nx, nv) in enumerate(shapes):
        pts = nx * nv
        per = nvg * R * (2 * Sv + 4) + nt * R * (2 * Sx + 2 * R)
        by = R + R
        if gi > 0:
            by += nvg * R / 2 ** d
        if gi + 1 < n:
            per += nxg * R * 4 + nt * R * (2 * Sv + 2 * R)
            by += nxg * R / 2 ** d
        flops += pts * per
        bytes_ += pts * by * elem_bytes
    return flops * B, bytes_ * B


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU execution is not implemented",
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
    prof = {name: ops.profile_read(slot) for slot, name in enumerate(["scan", "fused"])}
    ops.profile(False)
    ms_step = ms / a.steps
    value = B * ops.ndof / (ms_step * 1e-3)
    # dominant kernel
    dom = max(prof, key=lambda k: prof[k][0])
    fl, by = kernel_roofline(ops, ops.upper, B, R, 8 if a.dtype == "f64" else 4)
    fin_ms = prof["fused"][0] / max(prof["fused"][1], 1)
    ach_gbs = by / (fin_ms * 1e-3) / 1e9
    ach_tf = fl / (fin_ms * 1e-3) / 1e12
    t_hbm = by / (HBM_PEAK_GBS * 1e9)
    t_alu = fl / (FP64_VALU_PEAK_TFLOPS * 1e12)
    if t_alu > t_hbm:
        roof = {"bound": "alu", "achieved": round(ach_tf, 3), "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach_tf / FP64_VALU_PEAK_TFLOPS, 4), "traffic": None}
    else:
        roof = {"bound": "hbm", "achieved": round(ach_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach_gbs / HBM_PEAK_GBS, 4), "traffic": None}
    roof["kernel"] = "k_fused"
    roof["kernel_ms"] = round(fin_ms, 4)
    out = {
        "metric": "DOF-applies/s", "value": value, "unit": "DOF-applies/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": a.dtype, "data": "synthetic",
        "config": {"workload": f"4D phase space d=2, r=1, sparse grid L={a.level} (c2), full SD-DG operator",
                   "dofs_per_vector": ops.ndof, "batch": B, "grids": len(ops.upper)},
        "kernel_ms_per_step": {k: round(v[0] / a.steps, 4) for k, v in prof.items()},
        "dominant_kernel": dom,
        "roofline": roof,
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
    if not a.no_learned:
        out["learned"] = learned_leg(dev, a.train_steps)
    if a.batched > 0:
        out["batched"] = batched_leg(dev, a.batched)
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
    for name, mixed in (("fp64", False), ("mixed_fp32", True)):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = ops.solve_strip(b, x, sgdg.default_solve_opts(rtol=1e-8, mixed=mixed), raise_on_noconv=False)
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
    learned = sgdg.default_solve_opts(rtol=1e-8, maxit=400, pc=sgdg.default_precond_opts(net=net))
    learned_mixed = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True, pc=sgdg.default_precond_opts(net=net))
    for j in range(record_strips + 1, record_strips + test_strips + 1):
        b = ops.rhs(u, prev)
        row = {"strip": j}
        x, row["ct_fp64"] = _timed_solve(ops, b, ct)
        _, row["learned_fp64"] = _timed_solve(ops, b, learned)
        _, row["learned_mixed"] = _timed_solve(ops, b, learned_mixed)
        row["gain_learned_fp64"] = round(row["ct_fp64"]["seconds"] / row["learned_fp64"]["seconds"], 3)
        row["gain_learned_mixed"] = round(row["ct_fp64"]["seconds"] / row["learned_mixed"]["seconds"], 3)
        out["strips"].append(row)
        _log(f"learned leg: {row}")
        u = x
    net.close()
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
    seq, worst = 0.0, 0.0
    for ops, bb in zip(ops_list, bs):
        _, r = _timed_solve(ops, bb, sgdg.default_solve_opts(rtol=1e-8, maxit=400))
        seq += r["seconds"]
        worst = max(worst, r["rel_residual"])
    out["sequential_fp64_solve"] = {"seconds": round(seq, 3), "max_rel_residual": worst}
    out["speedup_batched_mixed_vs_sequential_fp64"] = round(seq / tb, 3)
    batch.close()
    for o in ops_list:
        o.close()
    return out


def _grids(shapes):
    return [(lx, lv) for lx, lv, _, _ in shapes]


def cpu_baseline(w, gpu_value):
    """The oracle (factored form, NumPy/SciPy FP64) on the host: single-vector applies."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle.operator import Problem
    from workloads import random_vector
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        P = Problem(w)
        u = random_vector(P.ndof, 0)[0]
        t0 = time.perf_counter()
        P.apply(u)   # first apply also builds the factor caches
        setup = time.perf_counter() - t0
        n = 0
        t0 = time.perf_counter()
        while n < 3 or (time.perf_counter() - t0 < 8.0 and n < 20):
            P.apply(u)
            n += 1
        el = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    v = n * P.ndof / el
    return {"value": v, "unit": "DOF-applies/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} single-vector applies of the same c2 operator after a {setup:.1f}s factor setup",
            "gpu_over_cpu": gpu_value / v}


if __name__ == "__main__":
    main()
