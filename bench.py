"""Benchmark: sparse-grid SD-DG operator application on one MI355X.

One step = one application of the full strip operator A^(delta) (all blocks
A_{l,l'} of every component-grid pair: per-grid Kronecker sweeps, cross-grid
level scans with the embedding matrices, term accumulation) to a batch of
synthetic input vectors already resident in HBM.  Workload (default): the 4D
phase-space problem (d=2, r=1, sparse-grid level 7, 620 892 space-time DOFs per
vector), 64 vectors (u and y, 636 MB in FP64, exceed the 256 MB MALL).

Prints one JSON line.  Beside the headline number:
  * timing: bracketed mean, per-step median and 10th/90th percentiles, and a
    cold run (a 512 MiB buffer written before each application);
  * roofline (the longest launch group) and roofline_apply (the whole
    application): algorithmic flops and compulsory bytes (u read, y written)
    against the FP64 vector and HBM peaks, frac = t_bound / t_measured;
  * apply_c2_legs: 1, 16 and 64 vectors in FP64, 1 and 64 in FP32;
  * strip_solve: the first strip of that problem solved to 1e-8 in FP64 and
    in mixed precision (FP32 inner, FP64 refinement), eagerly and with the
    grid-problem GMRES cycles replayed from captured graphs, with the Sect. 4.3
    Chebyshev mass inverses, and with inexact grid solves; strip_solve_small:
    strip 1 of the 4D problems at level 5 (the sizes the CPU oracle is timed on);
  * learned: the 4D Vlasov-type step (x periodic, frozen random E(x), L=7,
    r=0): (r, P_CT r) pairs recorded from CT-preconditioned solves of strips
    1-8, the per-grid networks trained on them, then strips 9-10 solved to 1e-8
    with CT, with the learned preconditioner, learned + mixed precision, and
    with inexact CT grid solves as CT and as the learned preconditioner's
    fallback; its "network" entry is the forward rate of the trained network
    with its matrix-core utilisation (--network-only: that rate alone);
  * batched_learned: four such problems (different fields), each with its own
    networks, solved in one batch with learned + mixed precision against the
    plain FP64 method one problem at a time;
  * batched: independent 4D problems with levels drawn from {5,6,7}, applied
    and solved in lockstep (FP32 applies inside FP64 refinement) against the
    same problems solved one at a time in plain FP64;
  * apply_6d: the 6D phase-space problem (d=3, L=6) applied to 1 and 8
    vectors in FP64 and 1 in FP32;
  * apply_2d: the 2D phase-space problem (d=1, L=6) applied to a batch, and
    its 8-strip march with CT-preconditioned FGMRES to 1e-10;
  * vlasov_poisson: Landau damping in 1+1 and 2+2 dimensions and the 1+1
    two-stream instability (with --twostream-2d also the 2+2 one over [0, 50],
    the run whose wall time the paper reports), the per-strip fixed point of
    transport and field, the electric energy and the two-stream growth rate;
  * table1: the periodic advection test of Sect. 5.1 (r = 1) for d = 1, 2, 3:
    every strip of one period solved on the device, the error in the SD norm
    and its observed order beside the paper's Table 1;
  * cpu_baseline: the CPU oracle timed on the host cores (one core and a
    process pool over all of them) on a bounded sample.
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
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--workload", choices=["c2", "c3"], default="c2",
                    help="operator of the timed apply: the 4D problem (default) or the 6D one")
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
    ap.add_argument("--no-vp", action="store_true", help="skip the Vlasov-Poisson leg")
    ap.add_argument("--vp-run", default="",
                    help="PROBLEM,D,LEVEL,DT,J0,J1: only strips J0..J1 of one Vlasov-Poisson run (landau or "
                         "twostream); J0 > 1 resumes from --vp-state, and the final state is written there")
    ap.add_argument("--vp-state", default="", help="state file (.npz) of --vp-run")
    ap.add_argument("--learned-run", type=int, default=0,
                    help="only the learned leg, with pairs recorded from this many CT-preconditioned strips")
    ap.add_argument("--twostream-2d", action="store_true",
                    help="add the 2+2-dimensional two-stream run at the paper's level 5 over [0, 50] (about 4 minutes)")
    ap.add_argument("--table1", default="6,6,3",
                    help="highest paper levels of the Table-1 leg for d = 1,2,3 (0 skips a dimension; 0 alone skips the leg)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--cold", type=int, default=10, help="cold-cache repetitions of the headline apply")
    ap.add_argument("--no-legs", action="store_true", help="skip the other batch sizes and dtypes of the 4D apply")
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
    Wd = {1: 5, 2: 19, 3: 65}[d]
    n = len(ops.upper)
    work = {k: [0.0, 0.0] for k in ("vstage", "ustage", "xstage", "fused", "scan")}
    # level scans (counted densely, every group at every lower point), per vector:
    # step t builds the partner sums of lower grid t (v-factor side) and of lower grid
    # nlow-1-t (x-factor side), R (2W + 4) flops per target point and group (the
    # restricted W-point stencil plus the two-parent recursion); the restriction
    # before step t >= 1 maps each group's previous array, R 2S flops per point.
    low = ops.lower
    nlow = len(low)
    pts = [nx * nv for _, _, nx, nv in low]
    for t in range(n - 1):
        for ng, lg in ((nvg, t), (nxg, nlow - 1 - t)):
            work["scan"][0] += B * pts[lg] * ng * R * (2 * Wd + 4)
            work["scan"][1] += B * pts[lg] * ng * R * elem_bytes      # the partner array written
            if t >= 1:
                rl = low[lg - 1][2] * low[lg][3] if lg == t else low[lg][2] * low[lg + 1][3]
                work["scan"][0] += B * rl * ng * R * 2 * S
                work["scan"][1] += B * rl * ng * R * elem_bytes
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
    summary of this workload, or None if there is none or the kernel source or the term
    builder changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"apply_{workload_tag}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    src = {"k_vstage": "split.hip", "k_ustage": "split.hip", "k_xstage": "split.hip", "k_xtile": "split.hip",
           "k_scan2": "fused.hip", "k_fused": "fused.hip"}.get(kernel)
    if src is None:
        return None
    text = open(path).read()
    # the counters hold for the kernel's source and for the term lists that set its work
    for f in (src, "terms.cpp"):
        sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2204_05988_amd", "csrc", f), "rb").read()).hexdigest()[:16]
        if f"{f} sha256/16 {sha}" not in text:
            return None
    for line in text.splitlines():
        f = line.split()
        if f and f[0] == kernel:
            return float(f[4])
    return None


def roofline(fl, by, ms, valu_peak):
    """Roofline position of a launch (or of a whole application) from its
    algorithmic flops `fl` and compulsory HBM bytes `by` in `ms` milliseconds:
    the bound is the larger of the two times at peak (VALU or HBM), and
    frac = t_bound / t_measured."""
    t_hbm = by / (HBM_PEAK_GBS * 1e9)
    t_alu = fl / (valu_peak * 1e12)
    t = ms * 1e-3
    if t_alu >= t_hbm:
        ach = fl / t / 1e12
        return {"bound": "alu", "achieved": round(ach, 3), "peak": valu_peak, "unit": "TFLOP/s",
                "frac": round(t_alu / t, 4), "hbm_frac_compulsory": round(by / t / 1e9 / HBM_PEAK_GBS, 4)}
    ach = by / t / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(t_hbm / t, 4), "alu_frac": round(fl / t / 1e12 / valu_peak, 4)}


SLOTS = {"scan": 0, "fused": 1, "vstage": 3, "ustage": 4, "xstage": 5}


def measure_apply(ops, B, dtname, steps, warmup, tune=True, cold=0, dev=None):
    """Times `steps` applications of the full operator to B vectors already in HBM.

    Returns the bracketed mean (events around all steps), the per-step median and
    10th/90th percentiles (events around each step), the per-kernel event times
    of the library (sgdg_profile, on the launching stream) and, with cold > 0,
    `cold` more steps each preceded by writing a 512 MiB buffer (the MALL holds
    256 MiB, so u, y and the tables come from HBM again)."""
    import torch
    from workloads import random_vector
    dt = torch.float64 if dtname == "f64" else torch.float32
    u = torch.tensor(random_vector(ops.ndof, 0, batch=B), device=dev, dtype=dt)
    y = torch.empty_like(u)
    stream = torch.cuda.current_stream()
    tuned = ops.tune(dtname, batch=B, reps=3) if tune else None
    for _ in range(warmup):
        ops.apply(u, y, batch=B)
    torch.cuda.synchronize()
    ops.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        ops.apply(u, y, batch=B)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    prof = {name: ops.profile_read(slot) for name, slot in SLOTS.items()}
    prof = {k: v for k, v in prof.items() if v[1] > 0}
    ops.profile(False)
    per = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ops.apply(u, y, batch=B)
        b.record(stream)
        b.synchronize()
        per.append(a.elapsed_time(b))
    out = {"batch": B, "dtype": dtname, "ms_mean": round(ms, 4), "ms_median": round(float(np.median(per)), 4),
           "ms_p10": round(float(np.percentile(per, 10)), 4), "ms_p90": round(float(np.percentile(per, 90)), 4),
           "dof_applies_per_s": B * ops.ndof / (ms * 1e-3), "launch_config": tuned, "wall_s": round(wall, 3),
           "kernel_ms_per_step": {k: round(v[0] / v[1] * (v[1] / steps), 4) for k, v in prof.items()}}
    if cold:
        junk = torch.empty(64 * 2 ** 20, dtype=torch.float64, device=dev)
        cms = []
        for _ in range(cold):
            junk.fill_(1.0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ops.apply(u, y, batch=B)
            b.record(stream)
            b.synchronize()
            cms.append(a.elapsed_time(b))
        out["cold"] = {"ms_median": round(float(np.median(cms)), 4), "ms_p10": round(float(np.percentile(cms, 10)), 4),
                       "ms_p90": round(float(np.percentile(cms, 90)), 4), "reps": cold,
                       "dof_applies_per_s": B * ops.ndof / (float(np.median(cms)) * 1e-3),
                       "note": "each application preceded by writing a 512 MiB buffer"}
        del junk
    return out, prof, tuned


def roofline_report(ops, B, dtname, prof, ms_step, tuned):
    """Per-kernel and whole-application roofline positions.

    Flops are the algorithmic counts of kernel_work.  Compulsory HBM bytes are
    those any implementation must move: u read once and y written once (the
    v-stage's u read and the last pass's y write); the design's own staged
    arrays (W between the passes, the partner scan arrays) are reported beside
    them as `bytes_staged`, not as algorithmic bytes."""
    R = ops.R
    elem = 8 if dtname == "f64" else 4
    valu_peak = FP64_VALU_PEAK_TFLOPS if dtname == "f64" else FP32_VALU_PEAK_TFLOPS
    work = kernel_work(ops, B, R, elem)
    io = B * ops.ndof * elem
    fused = tuned is not None and tuned.get("variant") == "fused"
    comp = {"vstage": io, "xstage": io, "ustage": 0, "scan": 0, "fused": 2 * io}
    per = {}
    for k, (tot, cnt) in prof.items():
        if k in work and cnt > 0:
            kms = tot / cnt
            # one event pair per launch group and application: the level scans are
            # 2 (grids - 1) - 1 launches of k_scan2, the other passes one launch each
            per[k] = dict(roofline(work[k][0], comp[k], kms, valu_peak), kernel_ms=round(kms, 4),
                          launches_in_group=2 * (len(ops.upper) - 1) - 1 if k == "scan" else 1,
                          flops=work[k][0], bytes_compulsory=comp[k], bytes_staged=work[k][1])
    kname = {k: "k_" + k for k in per}
    if "scan" in kname:
        kname["scan"] = "k_scan2"
    if tuned is not None and tuned.get("variant") == "split_tiled" and "xstage" in kname:
        kname["xstage"] = "k_xtile"
    used = ["scan", "fused"] if fused else ["scan", "vstage", "ustage", "xstage"]
    fl = sum(work[k][0] for k in used if k in work)
    whole = dict(roofline(fl, 2 * io, ms_step, valu_peak), ms=round(ms_step, 4), flops=fl,
                 flops_per_dof=round(fl / (B * ops.ndof), 1), bytes_compulsory=2 * io,
                 bytes_per_dof=2 * elem)
    return per, kname, whole


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; execution across several GPUs is not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.vp_run:
        print(json.dumps({"vp_run": vp_segment(a.vp_run, a.vp_state)}), flush=True)
        return
    import torch
    if a.learned_run:
        leg = learned_leg(torch.device("cuda:0"), a.train_steps, record_strips=a.learned_run)
        print(json.dumps({"learned_run": leg}), flush=True)
        return
    from paper_2204_05988_amd import sgdg
    from workloads import config_c2

    dev = torch.device("cuda:0")
    if a.workload == "c3":
        from workloads import config_c3
        w = config_c3(L=a.level if a.level != 7 else 6)
        wname = f"6D phase space d=3, r=0, sparse grid L={w.L} (c3), full SD-DG operator"
    else:
        w = config_c2(L=a.level)
        wname = f"4D phase space d=2, r=1, sparse grid L={a.level} (c2), full SD-DG operator"
    ops = sgdg.SparseGridOps(w)
    B = a.batch
    res, prof, tuned = measure_apply(ops, B, a.dtype, a.steps, a.warmup, tune=not a.no_tune, cold=a.cold, dev=dev)
    if tuned is not None:
        _log(f"launch configuration: {tuned}")
    ms_step = res["ms_mean"]
    value = res["dof_applies_per_s"]
    per_kernel, kname, whole = roofline_report(ops, B, a.dtype, prof, ms_step, tuned)
    dom = max(per_kernel, key=lambda k: per_kernel[k]["kernel_ms"])
    roof = dict(per_kernel[dom])
    roof["kernel"] = kname[dom]
    tag = f"{a.workload}_L{w.L}_B{B}_{a.dtype}"
    roof["traffic"] = recorded_traffic(kname[dom], tag)
    out = {
        "metric": "DOF-applies/s", "value": value, "unit": "DOF-applies/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": a.dtype, "data": "synthetic",
        "config": {"workload": wname,
                   "dofs_per_vector": ops.ndof, "batch": B, "grids": len(ops.upper)},
        "timing": {k: res[k] for k in ("ms_mean", "ms_median", "ms_p10", "ms_p90") if k in res},
        "kernel_ms_per_step": res["kernel_ms_per_step"],
        "launch_config": tuned,
        "dominant_kernel": kname[dom],
        "kernel_names": kname,
        "roofline": roof,
        "roofline_apply": whole,
        "kernels": per_kernel,
        "wall_s": res["wall_s"],
    }
    if "cold" in res:
        out["timing"]["cold"] = res["cold"]
    _log(f"apply: {value:.3e} DOF-applies/s, {ms_step:.4f} ms; whole-apply roofline {whole}")
    if a.calib_copy:
        src = torch.empty(64 * 2 ** 20, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        _log("calibration copy: 512 MiB read + 512 MiB written")
    if not a.no_legs:
        legs = {}
        combos = ((1, "f64"), (16, "f64"), (64, "f64"), (1, "f32"), (64, "f32")) if a.workload == "c2" else \
            ((1, "f64"), (8, "f64"), (1, "f32"))
        for Bl, dtl in combos:
            if Bl == B and dtl == a.dtype:
                continue
            r, p, t = measure_apply(ops, Bl, dtl, max(5, a.steps // 2), 2, tune=not a.no_tune, cold=5, dev=dev)
            pk, kn, wh = roofline_report(ops, Bl, dtl, p, r["ms_mean"], t)
            r["roofline_apply"] = wh
            r["kernels"] = {kn[k]: {"kernel_ms": v["kernel_ms"], "frac": v["frac"], "bound": v["bound"]}
                            for k, v in pk.items()}
            legs[f"{a.workload}_B{Bl}_{dtl}"] = r
            _log(f"{a.workload} leg B={Bl} {dtl}: {r['dof_applies_per_s']:.3e} DOF-applies/s, {r['ms_median']} ms median")
        out[f"apply_{a.workload}_legs"] = legs
    ops.close()
    gpu_strips = {}
    if not a.no_solve:
        ops = sgdg.SparseGridOps(w)
        out["strip_solve"] = solve_times(ops, w, dev)
        ops.close()
        _log(f"strip solves: {out['strip_solve']}")
        out["strip_solve_small"] = small_strips(dev)
        gpu_strips = {k: v["seconds"] for k, v in out["strip_solve_small"].items()}
    if a.network_only:
        out["network"] = network_leg(dev)
    elif not a.no_learned:
        out["learned"] = learned_leg(dev, a.train_steps)
        out["batched_learned"] = batched_learned_leg(dev)
    if a.batched > 0:
        out["batched"] = batched_leg(dev, a.batched)
    if not a.no_vp:
        runs = (("landau", 1, 5, 20), ("landau", 2, 5, 3), ("twostream", 1, 5, 100))
        if a.twostream_2d:
            runs = runs + (("twostream", 2, 5, 100),)
        out["vlasov_poisson"] = vlasov_poisson_leg(dev, runs)
    if a.c3_level > 0:
        out["apply_6d"] = apply_6d_leg(dev, a.c3_level)
    t1 = tuple((d + 1, int(m)) for d, m in enumerate(a.table1.split(",")) if m and int(m) > 0)
    if t1:
        out["table1"] = table1_leg(dev, t1)
    if not a.no_2d:
        out["apply_2d"] = apply_2d_leg(dev)
        gpu_strips.setdefault("c1_march", out["apply_2d"]["march"]["seconds"])
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, value, gpu_strips)
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
    # (grid preconditioner: mass diagonals, or 4 Chebyshev-Jacobi steps per mass factor;
    # graph: grid-problem GMRES cycles replayed from captured graphs, captured by a
    # preceding untimed solve)
    for name, mixed, cap, sweeps, graph in (("fp64", False, 200, 0, False), ("mixed_fp32", True, 200, 0, False),
                                            ("fp64_graph", False, 200, 0, True), ("mixed_fp32_graph", True, 200, 0, True),
                                            ("fp64_mass_cheb4", False, 200, 4, False),
                                            ("fp64_inexact_ct", False, 10, 0, False),
                                            ("mixed_fp32_inexact_ct", True, 10, 0, False)):
        opts = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=mixed, use_graph=graph,
                                       pc=sgdg.default_precond_opts(inner_maxit=cap, mass_sweeps=sweeps))
        if graph:
            ops.solve_strip(b, torch.zeros_like(b), opts, raise_on_noconv=False)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = ops.solve_strip(b, x, opts, raise_on_noconv=False)
        torch.cuda.synchronize()
        res[name] = {"seconds": round(time.perf_counter() - t0, 4), "outer_iters": st.outer_iters,
                     "inner_iters": st.inner_iters_total, "rel_residual": st.rel_residual,
                     "refinements": st.refinement_steps}
    return res


def _strip1_rhs(ops, w, dev):
    """b_1 on the device: U_0 the sparse-grid interpolant of u0, data f and g sampled
    at the strip's Gauss points (zero where the workload has none)."""
    import torch
    from workloads import gauss_legendre_times, sample_on_grids
    u0 = _interp_u0(ops, w, dev)
    tq, _ = gauss_legendre_times(0.0, w.dt, w.r + 2)

    def nodal(fn):
        if fn is None:
            return None
        return torch.tensor(np.stack([np.concatenate([sample_on_grids(w, _grids(ops.upper), fn, t),
                                                      sample_on_grids(w, _grids(ops.lower), fn, t)]) for t in tq]),
                            device=dev)

    return ops.rhs(u0, 1, nodal(w.f), nodal(w.g))


def small_strips(dev):
    """Strip 1 of the 4D problems at L = 5 (the sizes the CPU oracle is timed on),
    FP64 with the combination technique to 1e-8, eager and with the grid-problem
    GMRES cycles replayed from captured graphs."""
    from paper_2204_05988_amd import sgdg
    from workloads import config_c2, config_c5
    out = {}
    for name, w in (("c2_L5_strip1", config_c2(L=5)), ("c5_L5_strip1", config_c5(L=5))):
        ops = sgdg.SparseGridOps(w)
        b = _strip1_rhs(ops, w, dev)
        _timed_solve(ops, b, sgdg.default_solve_opts(rtol=1e-8, maxit=400))     # first use builds tables
        _, r = _timed_solve(ops, b, sgdg.default_solve_opts(rtol=1e-8, maxit=400))
        _timed_solve(ops, b, sgdg.default_solve_opts(rtol=1e-8, maxit=400, use_graph=True))   # captures
        _, rg = _timed_solve(ops, b, sgdg.default_solve_opts(rtol=1e-8, maxit=400, use_graph=True))
        out[name] = dict(r, dofs=ops.ndof, graph=rg)
        _log(f"small strip {name}: {out[name]}")
        ops.close()
    return out


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
    # the grid problems preconditioned by the x-transport inverse (periodic x, FFT) instead of
    # the mass diagonals: exact CT at a fraction of the inner iterations
    ct_transport = sgdg.default_solve_opts(rtol=1e-8, maxit=400, pc=sgdg.default_precond_opts(mass_sweeps=-2))
    ct_transport_mixed = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True,
                                                 pc=sgdg.default_precond_opts(mass_sweeps=-2))
    learned_transport = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True,
                                                pc=sgdg.default_precond_opts(net=net, mass_sweeps=-2))
    for j in range(record_strips + 1, record_strips + test_strips + 1):
        b = ops.rhs(u, prev)
        row = {"strip": j}
        x, row["ct_fp64"] = _timed_solve(ops, b, ct)
        _, row["ct_transport_fp64"] = _timed_solve(ops, b, ct_transport)
        _, row["ct_transport_mixed"] = _timed_solve(ops, b, ct_transport_mixed)
        _, row["learned_transport_fallback_mixed"] = _timed_solve(ops, b, learned_transport)
        _, row["learned_fp64"] = _timed_solve(ops, b, learned)
        _, row["learned_mixed"] = _timed_solve(ops, b, learned_mixed)
        _, row["ct_inexact_fp64"] = _timed_solve(ops, b, ct_inexact)
        _, row["learned_inexact_fallback_fp64"] = _timed_solve(ops, b, learned_inexact)
        _, row["learned_inexact_fallback_mixed"] = _timed_solve(ops, b, learned_inexact_mixed)
        t0 = row["ct_fp64"]["seconds"]
        row["gain_vs_ct_fp64"] = {k: round(t0 / row[k]["seconds"], 3)
                                  for k in ("learned_fp64", "learned_mixed", "ct_inexact_fp64",
                                            "learned_inexact_fallback_fp64", "learned_inexact_fallback_mixed",
                                            "ct_transport_fp64", "ct_transport_mixed",
                                            "learned_transport_fallback_mixed")}
        out["strips"].append(row)
        _log(f"learned leg: {row}")
        u = x
    net.close()
    ops.close()
    return out


def batched_learned_leg(dev, n=4, L=7, record_strips=8, train_steps=500):
    """Batched + learned + mixed precision against the plain FP64 method.

    n Vlasov-type problems (seeds 0..n-1: different fields E), each with its own
    networks trained on pairs recorded from its own CT-preconditioned solves of
    strips 1..record_strips; strip record_strips + 1 of every problem is then
    solved to 1e-8 (a) one problem at a time in FP64 with the combination
    technique, the plain method, and (b) all problems in one batch with the
    learned preconditioner, FP32 inner solves and FP64 refinement, once with
    the exact combination technique as the fallback and once with the inexact
    one (10 GMRES iterations per grid problem)."""
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import config_c5
    probs = []
    t0 = time.perf_counter()
    for seed in range(n):
        w = config_c5(seed=seed, L=L)
        ops = sgdg.SparseGridOps(w)
        net = sgdg.LearnedPreconditioner(ops, seed=seed)
        u = _interp_u0(ops, w, dev)
        net.record(4096)
        for j in range(1, record_strips + 1):
            b = ops.rhs(u, 1)
            u, _ = _timed_solve(ops, b, sgdg.default_solve_opts(rtol=1e-8, maxit=400))
        net.record(0)
        ts = net.train(train_steps, batch=8, lr=1e-3, seed=1)
        probs.append((w, ops, net, ops.rhs(u, 1), ts))
    prep = time.perf_counter() - t0
    out = {"workload": f"{n} Vlasov-type 4D problems (c5 fields, seeds 0..{n - 1}), L={L}, strip {record_strips + 1}",
           "problems": n, "dofs_total": sum(p[1].ndof for p in probs), "prep_s": round(prep, 2),
           "train": [{"pairs": p[2].pair_count(), "loss_first": p[4].loss_first, "loss_last": p[4].loss_last,
                      "seconds": round(p[4].seconds, 2)} for p in probs]}
    seq, worst = 0.0, 0.0
    for w, ops, net, b, _ in probs:
        _, r = _timed_solve(ops, b, sgdg.default_solve_opts(rtol=1e-8, maxit=400))
        seq += r["seconds"]
        worst = max(worst, r["rel_residual"])
    out["plain_fp64_one_at_a_time"] = {"seconds": round(seq, 4), "max_rel_residual": worst}
    batch = sgdg.SparseGridBatch([p[1] for p in probs])
    batch.set_networks([p[2] for p in probs])
    bt = torch.cat([p[3] for p in probs])
    for name, cap in (("batched_learned_mixed", 200), ("batched_learned_mixed_inexact_fallback", 10)):
        opts = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True,
                                       pc=sgdg.default_precond_opts(net=probs[0][2], inner_maxit=cap))
        batch.solve(bt, torch.zeros_like(bt), opts, raise_on_noconv=False)   # first use builds the batch tables
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, st = batch.solve(bt, torch.zeros_like(bt), opts, raise_on_noconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        out[name] = {"seconds": round(el, 4), "outer_iters": st.outer_iters, "refinements": st.refinement_steps,
                     "fallback": st.fallback_used, "pc_applications": st.pc_applications,
                     "max_rel_residual": st.rel_residual, "speedup_vs_plain_fp64": round(seq / el, 3)}
        _log(f"batched learned leg: {name} {out[name]}")
    for name, sweeps in (("batched_ct_mixed", 0), ("batched_ct_transport_mixed", -2)):
        opts = sgdg.default_solve_opts(rtol=1e-8, maxit=400, mixed=True,
                                       pc=sgdg.default_precond_opts(mass_sweeps=sweeps))
        batch.solve(bt, torch.zeros_like(bt), opts, raise_on_noconv=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, st = batch.solve(bt, torch.zeros_like(bt), opts, raise_on_noconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        out[name] = {"seconds": round(el, 4), "outer_iters": st.outer_iters, "inner_iters": st.inner_iters_total,
                     "max_rel_residual": st.rel_residual, "speedup_vs_plain_fp64": round(seq / el, 3)}
    _log(f"batched learned leg: {out}")
    batch.close()
    for p in probs:
        p[2].close()
        p[1].close()
    return out


def vlasov_poisson_leg(dev, runs=(("landau", 1, 5, 20), ("landau", 2, 5, 3), ("twostream", 1, 5, 100))):
    """Sect. 5.3 on the device, per run (problem, d, paper level, strips) with 0.5 time
    units per strip and r = 1: Landau damping (alpha = 0.01, k = 1/2, (0, 4 pi)^d x
    (-6, 6)^d) and the two-stream instability (alpha = 1e-3, k = 1/5, v0 = 2.4,
    (0, 10 pi)^d x (-9, 9)^d); the per-strip fixed point of transport and field,
    its electric energy, and for the two-stream runs the growth rate on [10, 20]
    beside the linear theory's 0.2258 (two Maxwellian beams, k = 1/5, v0 = 2.4)."""
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import config_landau, config_twostream
    out = {}
    for prob, d, pl, nst in runs:
        w = config_landau(d, pl) if prob == "landau" else config_twostream(d, pl)
        ops = sgdg.SparseGridOps(w)
        f = _interp_u0(ops, w, dev)
        ops.close()
        vp = sgdg.VlasovPoisson(w)
        E, en = vp.field(vp.density(f, 1))
        prev = 1
        energies, fps, secs, asm, outer = [en], [], [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vopts = sgdg.default_solve_opts(rtol=1e-10, pc=sgdg.default_precond_opts(mass_sweeps=-2))
        for j in range(nst):
            f, _, st = vp.strip(f, prev, E, fp_tol=1e-6, solve=vopts, raise_on_noconv=False)
            prev = w.r + 1
            E, en = vp.field(vp.density(f, prev, 1.0))
            energies.append(en)
            fps.append(st.fp_iters)
            secs.append(round(st.seconds, 4))
            asm.append(round(st.assemble_seconds, 4))
            outer.append(st.outer_iters)
            if (j + 1) % 10 == 0:
                _log(f"vlasov-poisson {prob} d={d}: strip {j + 1}/{nst}, energy {en:.3e}, "
                     f"{time.perf_counter() - t0:.1f}s")
        total = time.perf_counter() - t0
        key = f"{prob}_{d}d{d}v_paper_level{pl}"
        out[key] = {"dofs": vp.ndof, "x_nodes": vp.n_fine, "strips": nst, "t_end": nst * w.dt,
                    "seconds": round(total, 3), "fixed_point_iters": fps, "fgmres_iters": outer,
                    "strip_seconds": secs, "assemble_seconds": asm, "electric_energy": energies}
        if prob == "twostream" and nst * w.dt >= 20:
            t = np.arange(nst + 1) * w.dt
            keep = (t >= 10) & (t <= 20)
            out[key]["growth_rate_10_20"] = 0.5 * float(np.polyfit(t[keep], np.log(np.array(energies)[keep]), 1)[0])
            out[key]["growth_rate_linear_theory"] = 0.2258
        _log(f"vlasov-poisson {key}: {nst} strips in {total:.2f}s, fixed point {fps[:5]}...")
        vp.close()
    return out


def vp_segment(spec, state):
    """Strips J0..J1 of one Vlasov-Poisson run (spec "PROBLEM,D,LEVEL,DT,J0,J1"), the
    per-strip fixed point on the device; a run longer than one sitting is split into
    segments that hand over f, E and the energy history through the state file."""
    import torch
    from paper_2204_05988_amd import sgdg
    from workloads import config_landau, config_twostream
    prob, d, pl, dt, j0, j1 = spec.split(",")
    d, pl, dt, j0, j1 = int(d), int(pl), float(dt), int(j0), int(j1)
    w = (config_landau if prob == "landau" else config_twostream)(d, pl, dt=dt)
    dev = torch.device("cuda:0")
    vp = sgdg.VlasovPoisson(w)
    if j0 == 1:
        ops = sgdg.SparseGridOps(w)
        f = _interp_u0(ops, w, dev)
        ops.close()
        rho = vp.density(f, 1)
        E, en = vp.field(rho)
        prev, energies, masses, before = 1, [en], [float(rho.sum())], 0.0
    else:
        z = np.load(state)
        f = torch.tensor(z["f"], device=dev)
        E = torch.tensor(z["E"], device=dev)
        prev, energies, before = int(z["prev"]), list(z["energies"]), float(z["seconds"])
        # (a state written before the mass record existed resumes without it)
        masses = list(z["masses"]) if "masses" in z.files else []
        if len(energies) != j0:
            raise SystemExit(f"the state holds {len(energies) - 1} strips, not {j0 - 1}")
    vopts = sgdg.default_solve_opts(rtol=1e-10, pc=sgdg.default_precond_opts(mass_sweeps=-2))
    fps, outer, secs, asm = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(j0, j1 + 1):
        f, _, st = vp.strip(f, prev, E, fp_tol=1e-6, solve=vopts, raise_on_noconv=False)
        prev = w.r + 1
        rho = vp.density(f, prev, 1.0)
        E, en = vp.field(rho)
        energies.append(en)
        # the density summed over the periodic x-lattice is the mass up to a constant factor
        masses.append(float(rho.sum()))
        fps.append(st.fp_iters)
        outer.append(st.outer_iters)
        secs.append(round(st.seconds, 3))
        asm.append(round(st.assemble_seconds, 3))
        if (j - j0 + 1) % 10 == 0:
            _log(f"{prob} d={d} level {pl}: strip {j}/{j1}, t = {j * dt:g}, energy {en:.3e}, "
                 f"{time.perf_counter() - t0:.1f}s")
    seconds = time.perf_counter() - t0
    if state:
        np.savez(state, f=f.cpu().numpy(), E=E.cpu().numpy(), prev=prev, energies=np.array(energies),
                 masses=np.array(masses), seconds=before + seconds)
    out = {"problem": prob, "d": d, "paper_level": pl, "dt": dt, "strips": [j0, j1], "dofs": vp.ndof,
           "seconds": round(seconds, 2), "seconds_all_segments": round(before + seconds, 2),
           "fixed_point_iters": fps, "fgmres_iters": outer, "strip_seconds": secs, "assemble_seconds": asm,
           "electric_energy": energies,
           "mass_drift_max": (float(np.max(np.abs(np.array(masses) / masses[0] - 1)))
                              if len(masses) == len(energies) else None)}
    if prob == "landau":
        # damping rate of the field amplitude from the local maxima of the electric
        # energy (energy ~ exp(-2 gamma t)) up to t = 25, where the paper's runs
        # follow the linear rate
        t = np.arange(len(energies)) * dt
        e = np.array(energies)
        pk = [i for i in range(1, len(e) - 1) if e[i] >= e[i - 1] and e[i] >= e[i + 1] and t[i] <= 25]
        if len(pk) >= 3:
            out["decay_rate_0_25"] = -0.5 * float(np.polyfit(t[pk], np.log(e[pk]), 1)[0])
            out["decay_peaks"] = [[float(t[i]), float(e[i])] for i in pk]
    if prob == "twostream":
        t = np.arange(len(energies)) * dt
        keep = (t >= 10) & (t <= 20)
        if keep.sum() >= 3:
            out["growth_rate_10_20"] = 0.5 * float(np.polyfit(t[keep], np.log(np.array(energies)[keep]), 1)[0])
    vp.close()
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
    """Operator-apply throughput of the 6D phase-space problem (d=3, r=0): one and
    eight vectors in FP64, one in FP32, each with its whole-apply roofline."""
    from paper_2204_05988_amd import sgdg
    from workloads import config_c3
    w = config_c3(L=L)
    t0 = time.perf_counter()
    ops = sgdg.SparseGridOps(w)
    setup = time.perf_counter() - t0
    _log(f"6d leg: L={L}, {ops.ndof} DOFs, assembled in {setup:.1f}s")
    out = {"workload": f"6D phase space d=3, r=0, sparse grid L={L} (c3), full SD-DG operator", "dofs": ops.ndof,
           "grids": len(ops.upper), "setup_s": round(setup, 2)}
    for B, dt in ((1, "f64"), (8, "f64"), (1, "f32")):
        r, p, t = measure_apply(ops, B, dt, steps, 1, tune=True, cold=3, dev=dev)
        pk, kn, wh = roofline_report(ops, B, dt, p, r["ms_mean"], t)
        r["roofline_apply"] = wh
        r["kernels"] = {kn[k]: {"kernel_ms": v["kernel_ms"], "frac": v["frac"], "bound": v["bound"]}
                        for k, v in pk.items()}
        out[f"B{B}_{dt}"] = r
        _log(f"6d leg: B={B} {dt} {r['dof_applies_per_s']:.3e} DOF-applies/s, {r['ms_median']} ms median, "
             f"roofline {wh['frac']}")
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


# --- Sect. 5.1 (Table 1): the periodic advection test and its error in the SD norm -------------
#
# For beta = 1 in all 2d directions, sigma = 0 and periodic domains the strip
# operator satisfies, for every strip solution U (time slices U_s),
#   U^T A U = 1/2 ||U(t_j^-)||^2 + 1/2 ||U(t_{j-1}^+)||^2 + delta int_{I_j} ||d_t U + beta.grad U||^2
# (the mass-time-derivative and advection parts integrate to the trace terms,
# the advection part of a periodic constant-coefficient field vanishes, G^t
# adds the left trace).  The exact solution u solves d_t u + beta.grad u = 0
# and is continuous in time, so with e = U - u the norm (eq:norm_SD) is
#   |||e|||^2 = sum_j [U_j^T A U_j - (||U_j(t_j^-)||^2 + ||U_j(t_{j-1}^+)||^2) / 2]
#               + sum_{j<N} ||U_{j+1}(t_j^+) - U_j(t_j^-)||^2 + ||U_1(0^+) - u(0)||^2 + ||U_N(T^-) - u(T)||^2,
# every term an operator application or a mass product, the two end terms
# through ||w - u||^2 = ||w||^2 - 2 (u, w) + ||u||^2 with ||u||^2 = 1/2 and
# (u, phi_i (x) phi_j) = Im(exp(-4 pi i d t) a_lx a_lv exp(2 pi i sum x_i) exp(2 pi i sum v_j)),
# a_l the Fourier coefficient of the hat at the origin of the level-l lattice.

def _collapsed_rule(k, n):
    """Barycentric coordinates (Q, k+1) and weights (Q,) of a Gauss rule on the
    reference k-simplex (weights sum to 1/k!): a tensor Gauss-Legendre rule on
    the unit cube pushed through the collapsed (Duffy) coordinates."""
    g, gw = np.polynomial.legendre.leggauss(n)
    g, gw = 0.5 * (g + 1.0), 0.5 * gw
    mesh = np.stack(np.meshgrid(*([g] * k), indexing="ij"), -1).reshape(-1, k)
    wts = np.prod(np.stack(np.meshgrid(*([gw] * k), indexing="ij"), -1).reshape(-1, k), axis=1)
    y = np.empty_like(mesh)
    rest = np.ones(len(mesh))
    for j in range(k):
        y[:, j] = mesh[:, j] * rest
        rest = rest * (1.0 - mesh[:, j])
    jac = np.ones(len(mesh))
    for j in range(k - 1):
        jac *= (1.0 - mesh[:, j]) ** (k - 1 - j)
    bary = np.concatenate([1.0 - y.sum(axis=1, keepdims=True), y], axis=1)
    return bary, wts * jac


def hat_fourier(d, level, n=12):
    """int exp(2 pi i sum_a y_a) phi_0(y) dy, phi_0 the P1 hat at the origin of the
    level-`level` Kuhn lattice of the unit cube (spacing 2^-level).  Its support is
    the (d+1) d! simplices that have the origin as a vertex: for every ordering of
    the axes and every position k of the origin on the monotone path through a
    cell, the path shifted so that its k-th vertex is the origin."""
    import itertools
    h = 2.0 ** -level
    bary, wq = _collapsed_rule(d, n)
    tot = 0j
    for perm in itertools.permutations(range(d)):
        path = [np.zeros(d)]
        for a in perm:
            nxt = path[-1].copy()
            nxt[a] += 1.0
            path.append(nxt)
        path = np.array(path)
        for k in range(d + 1):
            pts = bary @ ((path - path[k]) * h)
            tot += h ** d * np.sum(wq * bary[:, k] * np.exp(2j * np.pi * pts.sum(axis=1)))
    return tot


def _exact_dot(w, grids, vec, t):
    """(u(t), W) for the Table-1 solution u and the one-slice spanning vector vec
    (host array) over the upper grids (lx, lv, nx, nv)."""
    from workloads import lattice_coords
    d = w.d
    out, off = 0.0, 0
    ph = np.exp(-4j * np.pi * d * t)
    for lx, lv, nx, nv in grids:
        ex = hat_fourier(d, lx) * np.exp(2j * np.pi * lattice_coords(w.x, lx).sum(axis=1))
        ev = hat_fourier(d, lv) * np.exp(2j * np.pi * lattice_coords(w.v, lv).sum(axis=1))
        blk = vec[off:off + nx * nv].reshape(nx, nv)
        out += float(np.imag(ph * (ex @ blk @ ev)))
        off += nx * nv
    return out


def sd_error_table1(w, grids, sols, apply_full, apply_mass, dot, cat, to_host):
    """SD-norm error of the strip solutions sols (each R slices on the upper grids
    (lx, lv, nx, nv)) of the Table-1 problem w, from operator applications only:
    apply_full(u) = A u, apply_mass(v) = M v (one slice); dot, cat and to_host act
    on the vectors' array type (numpy or device tensors)."""
    R = w.r + 1

    def traces(u):
        rt, lt, off = [], [], 0
        for _, _, nx, nv in grids:
            n = nx * nv
            blk = u[off:off + R * n].reshape(R, n)
            rt.append(blk.sum(0))
            lt.append(sum(((-1) ** s) * blk[s] for s in range(R)))
            off += R * n
        return cat(rt), cat(lt)

    sq = lambda v: dot(v, apply_mass(v))
    strip = jump = 0.0
    prev_right = None
    for j, u in enumerate(sols):
        right, left = traces(u)
        strip += dot(u, apply_full(u)) - 0.5 * (sq(right) + sq(left))
        if j == 0:
            first = left
        else:
            jump += sq(left - prev_right)
        prev_right = right
    T = len(sols) * w.dt
    end = 0.0
    for v, t in ((first, 0.0), (prev_right, T)):
        end += sq(v) - 2.0 * _exact_dot(w, grids, to_host(v), t) + 0.5
    return float(np.sqrt(strip + jump + end)), dict(strip=strip, jump=jump, end=end)


def table1_run(w, dev, tol=1e-10, mass_sweeps=0):
    """All 2^(Lp+1) strips of the Table-1 problem w on the device (FGMRES with the
    combination technique to tol), then the SD-norm error; returns (error, stats)."""
    import torch
    from paper_2204_05988_amd import sgdg
    ops = sgdg.SparseGridOps(w)
    t0 = time.perf_counter()
    u_prev, prev = _interp_u0(ops, w, dev), 1
    opts = sgdg.default_solve_opts(rtol=tol, maxit=400, pc=sgdg.default_precond_opts(mass_sweeps=mass_sweeps))
    sols, outer = [], 0
    for _ in range(w.nstrips):
        b = ops.rhs(u_prev, prev)
        u = torch.zeros_like(b)
        _, st = ops.solve_strip(b, u, opts)
        outer += st.outer_iters
        sols.append(u)
        u_prev, prev = u, ops.R
    torch.cuda.synchronize()
    march_s = time.perf_counter() - t0

    def full(u):
        y = torch.empty_like(u)
        ops.apply(u, y)
        return y

    def mass(v):
        y = torch.empty_like(v)
        ops.apply(v, y, kind=sgdg.OP_MASS)
        return y

    err, parts = sd_error_table1(w, ops.upper, sols, full, mass, lambda a, b: float(torch.dot(a, b)),
                                 torch.cat, lambda v: v.cpu().numpy())
    dim = ops.npts_up - ops.npts_low
    ops.close()
    return err, dict(dim=dim, strips=w.nstrips, outer_iters=outer, march_s=round(march_s, 3), parts=parts)


# Table 1 of the paper (Sect. 5.1), r = 1: SD-norm error after one period per paper level.
TABLE1_R1 = {1: {1: 8.68e-01, 2: 5.25e-01, 3: 2.03e-01, 4: 7.20e-02, 5: 2.55e-02, 6: 8.99e-03},
             2: {1: 8.14e-01, 2: 5.98e-01, 3: 2.64e-01, 4: 9.58e-02, 5: 3.39e-02, 6: 1.19e-02},
             3: {1: 7.36e-01, 2: 6.17e-01, 3: 3.13e-01, 4: 1.17e-01}}


def table1_leg(dev, levels=((1, 6), (2, 6), (3, 3))):
    """The r = 1 columns of Table 1 on the device: errors, observed orders and the
    paper's values beside them (P1 on Kuhn simplices here, the paper's d >= 2 runs
    use cubes)."""
    from workloads import config_table1
    out = {}
    for d, lmax in levels:
        rows, prev = [], None
        for Lp in range(1, lmax + 1):
            err, st = table1_run(config_table1(Lp, d=d), dev)
            row = dict(L=Lp, error=err, paper=TABLE1_R1[d].get(Lp), **st)
            if prev is not None:
                row["order"] = float(np.log2(prev / err))
            prev = err
            rows.append(row)
            _log(f"table 1 d={d} L={Lp}: dof {st['dim']} error {err:.3e} (paper {row['paper']}) "
                 f"order {row.get('order')} march {st['march_s']} s")
        out[f"d{d}"] = rows
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
