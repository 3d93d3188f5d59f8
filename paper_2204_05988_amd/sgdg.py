"""Python binding of libsgdg (ctypes).  Argument marshalling only: every step
of the method runs in the HIP library; PyTorch provides device memory and the
stream.  Raises if the library is not built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgdg.so")

OP_FULL, OP_BLOCKDIAG, OP_MASS, OP_DATA_F, OP_DATA_G = 0, 1, 2, 3, 4
F64, F32 = 0, 1
STATUS = {0: "OK", -1: "E_ARG", -2: "E_ALLOC", -3: "E_HIP", -4: "E_NOCONV", -5: "E_BREAKDOWN",
          -6: "E_NAN", -7: "E_STATE"}

EXPORTS = [
    "sgdg_last_error", "sgdg_build_sparse_grid", "sgdg_grid_info", "sgdg_grid_destroy",
    "sgdg_assemble_1d_factors", "sgdg_ops_destroy", "sgdg_apply_operator", "sgdg_combine",
    "sgdg_precondition", "sgdg_rhs", "sgdg_solve_strip", "sgdg_debug_dense_block",
    "sgdg_profile", "sgdg_profile_read", "sgdg_op_info", "sgdg_op_support",
    "sgdg_batch_create", "sgdg_batch_layout", "sgdg_batch_apply", "sgdg_batch_solve", "sgdg_batch_destroy",
    "sgdg_net_create", "sgdg_net_shape", "sgdg_net_get_params", "sgdg_net_set_params", "sgdg_net_add_pairs",
    "sgdg_net_record", "sgdg_net_pair_count", "sgdg_net_train", "sgdg_net_apply", "sgdg_net_forward",
    "sgdg_net_backward", "sgdg_net_destroy", "sgdg_tune", "sgdg_batch_tune", "sgdg_set_launch",
    "sgdg_graph_cache_size", "sgdg_debug_fallback", "sgdg_debug_grid_precond", "sgdg_apply_operator_noalloc",
    "sgdg_batch_set_networks", "sgdg_vp_create", "sgdg_vp_info", "sgdg_vp_density", "sgdg_vp_field",
    "sgdg_vp_strip", "sgdg_vp_destroy", "sgdg_assemble_factors_t",
]


class SgdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Domain(C.Structure):
    _fields_ = [("dim", C.c_int), ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("periodic", C.c_int)]


class Separable(C.Structure):
    _fields_ = [("scale", C.c_double), ("n_xf", C.c_int), ("xf", C.POINTER(C.POINTER(C.c_double))),
                ("n_vf", C.c_int), ("vf", C.POINTER(C.POINTER(C.c_double)))]


class Problem(C.Structure):
    _fields_ = [("beta", C.POINTER(Separable) * 6), ("n_sigma", C.c_int), ("sigma", C.POINTER(Separable)),
                ("dt", C.c_double), ("delta", C.c_double)]


class ProblemT(C.Structure):
    _fields_ = [("m", C.c_int), ("tau", C.POINTER(C.c_double)), ("weight", C.POINTER(C.c_double)),
                ("at", C.POINTER(Problem))]


class PrecondOpts(C.Structure):
    _fields_ = [("kind", C.c_int), ("inner_rtol", C.c_double), ("inner_maxit", C.c_int),
                ("inner_restart", C.c_int), ("mass_sweeps", C.c_int), ("net", C.c_void_p),
                ("fallback_iters", C.c_int), ("fallback_drop", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int), ("maxit", C.c_int), ("mixed_precision", C.c_int),
                ("inner_outer_rtol", C.c_double), ("pc", PrecondOpts), ("use_graph", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("refinement_steps", C.c_int), ("inner_iters_total", C.c_int),
                ("rel_residual", C.c_double), ("seconds", C.c_double), ("fallback_used", C.c_int),
                ("pc_applications", C.c_int)]


VARIANTS = ("split", "fused", "split_tiled")


class VpOpts(C.Structure):
    _fields_ = [("fp_tol", C.c_double), ("max_fp", C.c_int), ("solve", SolveOpts)]


class VpStats(C.Structure):
    _fields_ = [("fp_iters", C.c_int), ("outer_iters", C.c_int), ("inner_iters", C.c_int), ("dE", C.c_double),
                ("df", C.c_double), ("energy", C.c_double), ("rel_residual", C.c_double), ("seconds", C.c_double),
                ("assemble_seconds", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("variant", C.c_int), ("vectors_per_thread", C.c_int), ("xbox", C.c_int), ("block_map", C.c_int),
                ("ms", C.c_double), ("from_cache", C.c_int), ("scan_chunks", C.c_int)]

    def as_dict(self):
        return {"variant": VARIANTS[self.variant], "vectors_per_thread": self.vectors_per_thread,
                "xbox": self.xbox, "block_map": "xcd" if self.block_map else "round_robin", "ms": self.ms,
                "from_cache": bool(self.from_cache), "scan_chunks": self.scan_chunks}


class TrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("seed", C.c_uint64), ("mix", C.c_int)]


class TrainStats(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("seconds", C.c_double), ("steps", C.c_int)]


_LIB = None


def lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2204_05988_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64p, ip, dp = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_double)
    L.sgdg_last_error.restype = C.c_char_p
    L.sgdg_build_sparse_grid.argtypes = [C.POINTER(Domain), C.POINTER(Domain), C.c_int, C.c_int, C.c_int,
                                         C.POINTER(vp)]
    L.sgdg_grid_info.argtypes = [vp, C.c_int, ip, i64p, ip, ip, i64p, i64p, i64p]
    L.sgdg_grid_destroy.argtypes = [vp]
    L.sgdg_grid_destroy.restype = None
    L.sgdg_assemble_1d_factors.argtypes = [vp, C.POINTER(Problem), C.POINTER(vp)]
    L.sgdg_assemble_factors_t.argtypes = [vp, C.POINTER(ProblemT), C.POINTER(vp)]
    L.sgdg_ops_destroy.argtypes = [vp]
    L.sgdg_ops_destroy.restype = None
    L.sgdg_apply_operator.argtypes = [vp, C.c_int, vp, vp, C.c_int, C.c_int, vp]
    L.sgdg_apply_operator_noalloc.argtypes = [vp, C.c_int, vp, vp, C.c_int, C.c_int, vp]
    L.sgdg_combine.argtypes = [vp, vp, vp, C.c_int, vp]
    L.sgdg_precondition.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.POINTER(PrecondOpts), vp]
    L.sgdg_rhs.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp]
    L.sgdg_solve_strip.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp]
    L.sgdg_debug_dense_block.argtypes = [C.POINTER(Domain), C.POINTER(Domain), C.c_int, C.c_int, C.c_int,
                                         C.POINTER(Problem), C.c_int, C.c_int, C.c_int, dp]
    L.sgdg_profile.argtypes = [vp, C.c_int]
    L.sgdg_profile_read.argtypes = [vp, C.c_int, dp, i64p]
    L.sgdg_op_info.argtypes = [vp, C.c_int, ip, ip, ip, ip, ip, ip, ip]
    L.sgdg_op_support.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_int64)]
    L.sgdg_batch_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp)]
    L.sgdg_batch_layout.argtypes = [vp, i64p]
    L.sgdg_batch_apply.argtypes = [vp, vp, vp, C.c_int, vp]
    L.sgdg_batch_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp]
    L.sgdg_batch_set_networks.argtypes = [vp, C.POINTER(vp), C.c_int]
    L.sgdg_vp_create.argtypes = [vp, C.c_double, C.c_double, C.POINTER(vp)]
    L.sgdg_vp_info.argtypes = [vp, i64p, ip]
    L.sgdg_vp_density.argtypes = [vp, vp, C.c_int, C.c_double, vp, vp]
    L.sgdg_vp_field.argtypes = [vp, vp, vp, dp, vp]
    L.sgdg_vp_strip.argtypes = [vp, vp, C.c_int, vp, vp, vp, C.POINTER(VpOpts), C.POINTER(VpStats), vp]
    L.sgdg_vp_destroy.argtypes = [vp]
    L.sgdg_vp_destroy.restype = None
    L.sgdg_batch_destroy.argtypes = [vp]
    L.sgdg_batch_destroy.restype = None
    fp = C.POINTER(C.c_float)
    L.sgdg_net_create.argtypes = [vp, C.c_uint64, C.POINTER(vp)]
    L.sgdg_net_shape.argtypes = [vp, i64p, ip]
    L.sgdg_net_get_params.argtypes = [vp, fp, dp]
    L.sgdg_net_set_params.argtypes = [vp, fp, dp]
    L.sgdg_net_add_pairs.argtypes = [vp, vp, vp, C.c_int, vp]
    L.sgdg_net_record.argtypes = [vp, C.c_int]
    L.sgdg_net_pair_count.argtypes = [vp, ip]
    L.sgdg_net_train.argtypes = [vp, C.POINTER(TrainOpts), C.POINTER(TrainStats), vp]
    L.sgdg_net_apply.argtypes = [vp, vp, vp, vp]
    L.sgdg_net_forward.argtypes = [vp, vp, vp, vp]
    L.sgdg_net_backward.argtypes = [vp, vp, vp, vp, vp]
    L.sgdg_net_destroy.argtypes = [vp]
    L.sgdg_net_destroy.restype = None
    L.sgdg_tune.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(TuneResult), vp]
    L.sgdg_batch_tune.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(TuneResult), vp]
    L.sgdg_set_launch.argtypes = [vp, C.POINTER(TuneResult)]
    L.sgdg_graph_cache_size.argtypes = [vp, ip]
    L.sgdg_debug_fallback.argtypes = [C.c_int, C.c_double, C.c_int, ip, dp, dp, ip]
    L.sgdg_debug_grid_precond.argtypes = [vp, C.c_int, vp, vp, C.c_int, vp]
    for name in EXPORTS:
        if name not in ("sgdg_last_error", "sgdg_grid_destroy", "sgdg_ops_destroy", "sgdg_batch_destroy",
                        "sgdg_net_destroy", "sgdg_vp_destroy"):
            getattr(L, name).restype = C.c_int
    _LIB = L
    return L


def _check(code):
    if code != 0:
        raise SgdgError(code, lib().sgdg_last_error().decode())


def _domain(dom) -> Domain:
    d = Domain()
    d.dim = dom.d
    for a in range(3):
        d.lo[a] = dom.lo[a] if a < dom.d else 0.0
        d.hi[a] = dom.hi[a] if a < dom.d else 1.0
    d.periodic = int(dom.periodic)
    return d


class _ProblemHolder:
    """Builds the C problem struct from a workload; keeps every array alive."""

    def __init__(self, w, fx, fv):
        self.keep = []
        self.p = Problem()

        def arr(a):
            a = np.ascontiguousarray(a, dtype=np.float64)
            self.keep.append(a)
            return a.ctypes.data_as(C.POINTER(C.c_double))

        def sep(scale, xn, vn):
            s = Separable()
            s.scale = float(scale)
            xs = (C.POINTER(C.c_double) * max(1, len(xn)))(*[arr(fx[k]) for k in xn])
            vs = (C.POINTER(C.c_double) * max(1, len(vn)))(*[arr(fv[k]) for k in vn])
            self.keep += [xs, vs]
            s.n_xf, s.xf = len(xn), C.cast(xs, C.POINTER(C.POINTER(C.c_double)))
            s.n_vf, s.vf = len(vn), C.cast(vs, C.POINTER(C.POINTER(C.c_double)))
            self.keep.append(s)
            return s

        for c in range(6):
            b = w.beta[c] if c < len(w.beta) else None
            self.p.beta[c] = C.pointer(sep(*b)) if b is not None else C.POINTER(Separable)()
        sig = (Separable * max(1, len(w.sigma)))()
        for i, (sc, P, Q) in enumerate(w.sigma):
            sig[i] = sep(sc, P, Q)
        self.keep.append(sig)
        self.p.n_sigma = len(w.sigma)
        self.p.sigma = C.cast(sig, C.POINTER(Separable))
        self.p.dt = w.dt
        self.p.delta = w.delta


def _ptr(t) -> int:
    return t.data_ptr()


def _dev(t, name, numel, dtypes=("float64",)):
    """Checks one device-buffer argument before any launch: a contiguous GPU
    tensor of an accepted dtype holding exactly `numel` elements.  A wrong
    buffer would otherwise become an out-of-bounds device access."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if str(t.dtype).replace("torch.", "") not in dtypes:
        raise TypeError(f"{name}: dtype {t.dtype} not in {dtypes}")
    if t.numel() != numel:
        raise ValueError(f"{name}: has {t.numel()} elements, expected {numel}")
    return t.data_ptr()


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def default_precond_opts(inner_rtol=1e-8, inner_maxit=200, inner_restart=30, mass_sweeps=0, net=None,
                         fallback_iters=10, fallback_drop=10.0) -> PrecondOpts:
    """kind 0 (combination technique), or kind 1 (learned) when a LearnedPreconditioner is given."""
    return PrecondOpts(1 if net is not None else 0, inner_rtol, inner_maxit, inner_restart, mass_sweeps,
                       net.h if net is not None else None, fallback_iters, fallback_drop)


def default_solve_opts(rtol=1e-8, restart=50, maxit=400, mixed=False, inner_outer_rtol=1e-4, pc=None,
                       use_graph=False) -> SolveOpts:
    return SolveOpts(rtol, restart, maxit, int(mixed), inner_outer_rtol, pc or default_precond_opts(),
                     int(use_graph))


class SparseGridOps:
    """One strip operator of a workload on the current HIP device."""

    def __init__(self, w, fields=None, t0=0.0):
        """w.tfields set: coefficients that depend on time, sampled at the w.tquad
        (default r + 2) Gauss-Legendre points of the strip [t0, t0 + dt]."""
        from workloads import lattice_coords, nodal_fields
        L = lib()
        self.w = w
        self.R = w.r + 1
        fx, fv = fields if fields is not None else nodal_fields(w)
        self._dx, self._dv = _domain(w.x), _domain(w.v)
        g = C.c_void_p()
        _check(L.sgdg_build_sparse_grid(C.byref(self._dx), C.byref(self._dv), w.lmin, w.L, w.r, C.byref(g)))
        self.grid = g
        o = C.c_void_p()
        if w.tfields is None:
            self.prob = _ProblemHolder(w, fx, fv)
            _check(L.sgdg_assemble_1d_factors(g, C.byref(self.prob.p), C.byref(o)))
        else:
            m = w.tquad if w.tquad else w.r + 2
            tau, wts = np.polynomial.legendre.leggauss(m)
            X, V = lattice_coords(w.x, w.L), lattice_coords(w.v, w.L)
            self.prob = []
            for t in t0 + 0.5 * w.dt * (tau + 1.0):
                xf, vf = w.tfields(t)
                self.prob.append(_ProblemHolder(w, {k: fn(X) for k, fn in xf.items()},
                                                {k: fn(V) for k, fn in vf.items()}))
            at = (Problem * m)(*[h.p for h in self.prob])
            self._t = (np.ascontiguousarray(tau), np.ascontiguousarray(wts), at)
            pt = ProblemT(m, self._t[0].ctypes.data_as(C.POINTER(C.c_double)),
                          self._t[1].ctypes.data_as(C.POINTER(C.c_double)), C.cast(at, C.POINTER(Problem)))
            _check(L.sgdg_assemble_factors_t(g, C.byref(pt), C.byref(o)))
        self.ops = o
        self.upper = self.info(0)
        self.lower = self.info(1)
        self.ndof = int(self.R * sum(nx * nv for _, _, nx, nv in self.upper))
        self.npts_up = int(sum(nx * nv for _, _, nx, nv in self.upper))
        self.npts_low = int(sum(nx * nv for _, _, nx, nv in self.lower))

    def info(self, which):
        L = lib()
        n = C.c_int()
        _check(L.sgdg_grid_info(self.grid, which, C.byref(n), None, None, None, None, None, None))
        k = n.value
        lx, lv = (C.c_int * max(k, 1))(), (C.c_int * max(k, 1))()
        nx, nv = (C.c_int64 * max(k, 1))(), (C.c_int64 * max(k, 1))()
        _check(L.sgdg_grid_info(self.grid, which, None, None, lx, lv, nx, nv, None))
        return [(lx[i], lv[i], nx[i], nv[i]) for i in range(k)]

    def close(self):
        if getattr(self, "ops", None):
            lib().sgdg_ops_destroy(self.ops)
            self.ops = None
        if getattr(self, "grid", None):
            lib().sgdg_grid_destroy(self.grid)
            self.grid = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- calls -------------------------------------------------------------------
    def apply(self, u, y, kind=OP_FULL, batch=1, stream=None):
        import torch
        n = self.ndof // self.R if kind == OP_MASS else self.ndof
        pu = _dev(u, "u", batch * n, ("float64", "float32"))
        py = _dev(y, "y", batch * n, (str(u.dtype).replace("torch.", ""),))
        dt = F64 if u.dtype == torch.float64 else F32
        _check(lib().sgdg_apply_operator(self.ops, kind, pu, py, dt, batch, _stream(stream)))
        return y

    def apply_noalloc(self, u, y, kind=OP_FULL, batch=1, stream=None):
        """The same operator through sgdg_apply_operator_noalloc (scratch from the
        library's fixed device array; the tables must exist: apply() once first)."""
        import torch
        n = self.ndof // self.R if kind == OP_MASS else self.ndof
        pu = _dev(u, "u", batch * n, ("float64", "float32"))
        py = _dev(y, "y", batch * n, (str(u.dtype).replace("torch.", ""),))
        dt = F64 if u.dtype == torch.float64 else F32
        _check(lib().sgdg_apply_operator_noalloc(self.ops, kind, pu, py, dt, batch, _stream(stream)))
        return y

    def combine(self, nodal, coef, nslices, stream=None):
        pn = _dev(nodal, "nodal", nslices * (self.npts_up + self.npts_low))
        pc = _dev(coef, "coef", nslices * self.npts_up)
        _check(lib().sgdg_combine(self.ops, pn, pc, nslices, _stream(stream)))
        return coef

    def precondition(self, r, z, opts: Optional[PrecondOpts] = None, stream=None, batch=1):
        import torch
        assert batch >= 1
        pr = _dev(r, "r", batch * self.ndof, ("float64", "float32"))
        pz = _dev(z, "z", batch * self.ndof, (str(r.dtype).replace("torch.", ""),))
        dt = F64 if r.dtype == torch.float64 else F32
        o = opts or default_precond_opts()
        _check(lib().sgdg_precondition(self.ops, pr, pz, dt, batch, C.byref(o), _stream(stream)))
        return z

    def rhs(self, u_prev, prev_slices, f_nodal=None, g_nodal=None, b=None, stream=None):
        import torch
        if b is None:
            b = torch.empty(self.ndof, dtype=torch.float64, device=u_prev.device)
        pu = _dev(u_prev, "u_prev", prev_slices * self.npts_up)
        nq = self.w.r + 2
        nn = nq * (self.npts_up + self.npts_low)
        pf = _dev(f_nodal, "f_nodal", nn) if f_nodal is not None else None
        pg = _dev(g_nodal, "g_nodal", nn) if g_nodal is not None else None
        pb = _dev(b, "b", self.ndof)
        _check(lib().sgdg_rhs(self.ops, pu, prev_slices, pf, pg, pb, _stream(stream)))
        return b

    def profile(self, on: bool):
        _check(lib().sgdg_profile(self.ops, 1 if on else 0))

    def profile_read(self, slot):
        ms, n = C.c_double(), C.c_int64()
        _check(lib().sgdg_profile_read(self.ops, slot, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def op_info(self, kind=OP_FULL):
        v = [C.c_int() for _ in range(7)]
        _check(lib().sgdg_op_info(self.ops, kind, *[C.byref(x) for x in v]))
        return dict(zip(["nterms", "nvg", "nxg", "Sx", "Sv", "Rin", "Rout"], [x.value for x in v]))

    def op_support(self, lx, kind=OP_FULL):
        """Per x-level support counts of the X-factors (see sgdg_op_support)."""
        c = (C.c_int64 * 6)()
        _check(lib().sgdg_op_support(self.ops, kind, lx, c))
        return dict(zip(["nodes", "read_groups", "read_terms", "row_groups", "qt_groups", "qt_terms"], list(c)))

    def tune(self, dtype="f64", batch=1, reps=3, force=False, stream=None):
        """Pick the fastest launch configuration of the full apply (cached on disk)."""
        r = TuneResult()
        _check(lib().sgdg_tune(self.ops, F64 if dtype == "f64" else F32, batch, reps, int(force), C.byref(r),
                               _stream(stream)))
        return r.as_dict()

    def set_launch(self, variant="split", vectors_per_thread=2, xbox=8, block_map=0, scan_chunks=0):
        r = TuneResult(VARIANTS.index(variant), vectors_per_thread, xbox, block_map, 0.0, 0, scan_chunks)
        _check(lib().sgdg_set_launch(self.ops, C.byref(r)))

    def grid_precond(self, x, y, sweeps=0, stream=None):
        """Diagnostic: the grid-problem preconditioner on the layout of every
        upper grid followed by every lower grid ([R][n_x][n_v] blocks)."""
        import torch
        n = self.R * (self.npts_up + self.npts_low)
        px = _dev(x, "x", n, ("float64", "float32"))
        py = _dev(y, "y", n, (str(x.dtype).replace("torch.", ""),))
        _check(lib().sgdg_debug_grid_precond(self.ops, sweeps, px, py, F64 if x.dtype == torch.float64 else F32,
                                             _stream(stream)))
        return y

    def graph_cache_size(self):
        c = C.c_int()
        _check(lib().sgdg_graph_cache_size(self.ops, C.byref(c)))
        return c.value

    def solve_strip(self, b, u, opts: Optional[SolveOpts] = None, stream=None, raise_on_noconv=True):
        pb = _dev(b, "b", self.ndof)
        pu = _dev(u, "u", self.ndof)
        o = opts or default_solve_opts()
        st = SolveStats()
        code = lib().sgdg_solve_strip(self.ops, pb, pu, C.byref(o), C.byref(st), _stream(stream))
        if code != 0 and (raise_on_noconv or code != -4):
            _check(code)
        return u, st


class SparseGridBatch:
    """Independent strip problems applied and solved together (one launch per
    kernel for the whole batch).  Vectors are the concatenation of the
    problems' vectors, problem i at offsets[i]."""

    def __init__(self, ops_list):
        L = lib()
        self.members = list(ops_list)  # keeps the ops handles alive
        arr = (C.c_void_p * len(self.members))(*[m.ops.value for m in self.members])
        h = C.c_void_p()
        _check(L.sgdg_batch_create(arr, len(self.members), C.byref(h)))
        self.h = h
        off = (C.c_int64 * (len(self.members) + 1))()
        _check(L.sgdg_batch_layout(h, off))
        self.offsets = [int(off[i]) for i in range(len(self.members) + 1)]
        self.ndof = self.offsets[-1]

    def apply(self, u, y, stream=None):
        import torch
        pu = _dev(u, "u", self.ndof, ("float64", "float32"))
        py = _dev(y, "y", self.ndof, (str(u.dtype).replace("torch.", ""),))
        dt = F64 if u.dtype == torch.float64 else F32
        _check(lib().sgdg_batch_apply(self.h, pu, py, dt, _stream(stream)))
        return y

    def tune(self, dtype="f64", reps=3, force=False, stream=None):
        r = TuneResult()
        _check(lib().sgdg_batch_tune(self.h, F64 if dtype == "f64" else F32, reps, int(force), C.byref(r),
                                     _stream(stream)))
        return r.as_dict()

    def solve(self, b, u, opts: Optional[SolveOpts] = None, stream=None, raise_on_noconv=True):
        pb = _dev(b, "b", self.ndof)
        pu = _dev(u, "u", self.ndof)
        o = opts or default_solve_opts()
        st = SolveStats()
        code = lib().sgdg_batch_solve(self.h, pb, pu, C.byref(o), C.byref(st), _stream(stream))
        if code != 0 and (raise_on_noconv or code != -4):
            _check(code)
        return u, st

    def set_networks(self, nets):
        """One LearnedPreconditioner per problem (same order), used by solves with
        a learned preconditioner (default_precond_opts(net=...) with any of them);
        an empty list removes them."""
        arr = (C.c_void_p * max(1, len(nets)))(*[n.h.value for n in nets])
        _check(lib().sgdg_batch_set_networks(self.h, arr, len(nets)))
        self._nets = list(nets)  # keeps the networks alive

    def close(self):
        if getattr(self, "h", None):
            lib().sgdg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LearnedPreconditioner:
    """The per-grid correction networks of one problem (d = 2)."""

    def __init__(self, ops: SparseGridOps, seed=0):
        L = lib()
        self.ops = ops  # keeps the problem alive
        h = C.c_void_p()
        _check(L.sgdg_net_create(ops.ops, seed, C.byref(h)))
        self.h = h
        n, g = C.c_int64(), C.c_int()
        _check(L.sgdg_net_shape(h, C.byref(n), C.byref(g)))
        self.n_params, self.n_grids = n.value, g.value

    def get_params(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        sc = np.zeros(self.n_grids)
        _check(lib().sgdg_net_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                         sc.ctypes.data_as(C.POINTER(C.c_double))))
        return p, sc

    def set_params(self, params=None, scales=None):
        pp = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        ss = None if scales is None else np.ascontiguousarray(scales, dtype=np.float64)
        _check(lib().sgdg_net_set_params(self.h, None if pp is None else pp.ctypes.data_as(C.POINTER(C.c_float)),
                                         None if ss is None else ss.ctypes.data_as(C.POINTER(C.c_double))))

    def add_pairs(self, r, z, stream=None):
        assert r.numel() % self.ops.ndof == 0 and r.numel() > 0
        pr = _dev(r, "r", r.numel())
        pz = _dev(z, "z", r.numel())
        _check(lib().sgdg_net_add_pairs(self.h, pr, pz, r.numel() // self.ops.ndof, _stream(stream)))

    def record(self, capacity):
        _check(lib().sgdg_net_record(self.h, capacity))

    def pair_count(self):
        c = C.c_int()
        _check(lib().sgdg_net_pair_count(self.h, C.byref(c)))
        return c.value

    def train(self, steps, batch=8, lr=1e-3, seed=0, mix=True, stream=None):
        o = TrainOpts(steps, batch, lr, seed, int(mix))
        st = TrainStats()
        _check(lib().sgdg_net_train(self.h, C.byref(o), C.byref(st), _stream(stream)))
        return st

    def apply(self, r, z, stream=None):
        pr = _dev(r, "r", self.ops.ndof)
        pz = _dev(z, "z", self.ops.ndof)
        _check(lib().sgdg_net_apply(self.h, pr, pz, _stream(stream)))
        return z

    def forward(self, x, y, stream=None):
        px = _dev(x, "x", self.ops.ndof, ("float32",))
        py = _dev(y, "y", self.ops.ndof, ("float32",))
        _check(lib().sgdg_net_forward(self.h, px, py, _stream(stream)))
        return y

    def backward(self, x, dy, grad, stream=None):
        px = _dev(x, "x", self.ops.ndof, ("float32",))
        pd = _dev(dy, "dy", self.ops.ndof, ("float32",))
        pg = _dev(grad, "grad", self.n_params, ("float32",))
        _check(lib().sgdg_net_backward(self.h, px, pd, pg, _stream(stream)))
        return grad

    def close(self):
        if getattr(self, "h", None):
            lib().sgdg_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VlasovPoisson:
    """The Vlasov-Poisson fixed point on a workload's sparse-grid layout (x
    periodic, d <= 2): density, field and strips, all on the device."""

    def __init__(self, w):
        L = lib()
        self.w = w
        self.R = w.r + 1
        self._dx, self._dv = _domain(w.x), _domain(w.v)
        g = C.c_void_p()
        _check(L.sgdg_build_sparse_grid(C.byref(self._dx), C.byref(self._dv), w.lmin, w.L, w.r, C.byref(g)))
        self.grid = g
        h = C.c_void_p()
        _check(L.sgdg_vp_create(g, w.dt, w.delta, C.byref(h)))
        self.h = h
        n, d = C.c_int64(), C.c_int()
        _check(L.sgdg_vp_info(h, C.byref(n), C.byref(d)))
        self.n_fine, self.d = n.value, d.value
        k = C.c_int()
        _check(L.sgdg_grid_info(g, 0, C.byref(k), None, None, None, None, None, None))
        nx, nv = (C.c_int64 * k.value)(), (C.c_int64 * k.value)()
        _check(L.sgdg_grid_info(g, 0, None, None, None, None, nx, nv, None))
        self.npts = int(sum(a * b for a, b in zip(nx, nv)))
        self.ndof = self.R * self.npts

    def density(self, f, nslices, tau=0.0, rho=None, stream=None):
        import torch
        if rho is None:
            rho = torch.empty(self.n_fine, dtype=torch.float64, device=f.device)
        pf = _dev(f, "f", nslices * self.npts)
        pr = _dev(rho, "rho", self.n_fine)
        _check(lib().sgdg_vp_density(self.h, pf, nslices, tau, pr, _stream(stream)))
        return rho

    def field(self, rho, E=None, stream=None):
        """(E [d][n_fine], electric energy)."""
        import torch
        if E is None:
            E = torch.empty(self.d * self.n_fine, dtype=torch.float64, device=rho.device)
        en = C.c_double()
        _check(lib().sgdg_vp_field(self.h, _dev(rho, "rho", self.n_fine), _dev(E, "E", self.d * self.n_fine),
                                   C.byref(en), _stream(stream)))
        return E, en.value

    def strip(self, f_prev, prev_slices, E0, fp_tol=1e-9, max_fp=30, solve=None, stream=None,
              raise_on_noconv=True):
        """(f, E, stats) of one strip of the fixed point."""
        import torch
        f = torch.empty(self.ndof, dtype=torch.float64, device=f_prev.device)
        E = torch.empty(self.d * self.n_fine, dtype=torch.float64, device=f_prev.device)
        o = VpOpts(fp_tol, max_fp, solve or default_solve_opts(rtol=1e-10))
        st = VpStats()
        code = lib().sgdg_vp_strip(self.h, _dev(f_prev, "f_prev", prev_slices * self.npts), prev_slices,
                                   _dev(E0, "E0", self.d * self.n_fine), _dev(f, "f", self.ndof),
                                   _dev(E, "E", self.d * self.n_fine), C.byref(o), C.byref(st), _stream(stream))
        if code != 0 and (raise_on_noconv or code != -4):
            _check(code)
        return f, E, st

    def close(self):
        if getattr(self, "h", None):
            lib().sgdg_vp_destroy(self.h)
            self.h = None
        if getattr(self, "grid", None):
            lib().sgdg_grid_destroy(self.grid)
            self.grid = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_dense_block(w, kind, row_grid, col_grid, fields=None):
    """Host-only dense operator block from the library's host assembly (diagnostics)."""
    from workloads import grid_levels, lattice_shape, nodal_fields
    fx, fv = fields if fields is not None else nodal_fields(w)
    holder = _ProblemHolder(w, fx, fv)
    up, _ = grid_levels(w)
    R = w.r + 1
    Rin = Rout = 1 if kind == OP_MASS else R
    n = lambda dom, l: int(np.prod(lattice_shape(dom, l)))
    (lx, lv), (lx2, lv2) = up[row_grid], up[col_grid]
    rows, cols = Rout * n(w.x, lx) * n(w.v, lv), Rin * n(w.x, lx2) * n(w.v, lv2)
    out = np.zeros((rows, cols))
    dx, dv = _domain(w.x), _domain(w.v)
    _check(lib().sgdg_debug_dense_block(C.byref(dx), C.byref(dv), w.lmin, w.L, w.r, C.byref(holder.p), kind,
                                        row_grid, col_grid, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def debug_fallback(iters, drop, calls, rel0, est):
    """Host-only: index of the FGMRES iteration after which the learned
    preconditioner's fallback rule switches to the combination technique (-1: never)."""
    n = len(est)
    ca = np.ascontiguousarray(calls, dtype=np.int32)
    ra = np.ascontiguousarray(rel0, dtype=np.float64)
    ea = np.ascontiguousarray(est, dtype=np.float64)
    out = C.c_int()
    _check(lib().sgdg_debug_fallback(int(iters), float(drop), n, ca.ctypes.data_as(C.POINTER(C.c_int)),
                                     ra.ctypes.data_as(C.POINTER(C.c_double)),
                                     ea.ctypes.data_as(C.POINTER(C.c_double)), C.byref(out)))
    return out.value
