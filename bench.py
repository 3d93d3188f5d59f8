"""Benchmark: sparse-grid SD-DG operator application on one MI355X.

One step = one application of the full strip operator A^(delta) (all blocks
A_{l,l'} of every component-grid pair: per-grid Kronecker sweeps, cross-grid
level scans with the embedding matrices, term accumulation) to a batch of
synthetic input vectors already resident in HBM.  Workload: the 4D phase-space
problem (d=2, r=1, sparse-grid level 7, 620 892 space-time DOFs per vector).

Prints one JSON line (rank 0).  Also reports, beside the headline number, the
strip-solve time to 1e-8 in FP64 and in mixed precision, and the CPU oracle
timed on a bounded sample.
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
    if not a.no_solve:
        out["strip_solve"] = solve_times(ops, w, dev)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, value)
    print(json.dumps(out), flush=True)


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
