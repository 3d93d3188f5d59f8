"""Workload definitions: the phase-space transport problems the method is run on.

Every workload is a linear transport problem in phase space (x, v), with
x in a d-dimensional box and v in a d-dimensional box (Sect. 1 of the paper,
problem (eq:transport)/(eq:inflow)).  Coefficients are given in the separable
form of Sect. 4.2: each component of beta is ONE product a(x)*b(v), sigma is a
short sum of products p(x)*q(v).  Each factor a, b, p, q is a product of named
fields; a named field is sampled at the lattice nodes of the finest level of its
domain (P1 nodal values).  Analytic data (u0, f, g) are plain numpy callables.

Lattice convention (shared by both implementations, it is the data layout):
level l of a box has 2**l cells per axis; nodes are numbered in C order over
the axis indices (the last axis varies fastest); a periodic axis has 2**l
nodes, a non-periodic one 2**l + 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

__all__ = [
    "Domain", "Workload", "lattice_shape", "lattice_coords", "nodal_fields",
    "grid_levels", "gauss_legendre_times", "random_vector", "sample_on_grids",
    "config_c1", "config_c2", "config_c3", "config_c4_member", "config_c4",
    "config_c5", "config_table1", "config_tiny", "config_landau", "config_twostream", "config_timedep_exact",
    "with_time_fields", "h_min",
]


@dataclasses.dataclass(frozen=True)
class Domain:
    d: int
    lo: tuple
    hi: tuple
    periodic: bool = False


@dataclasses.dataclass
class Workload:
    name: str
    x: Domain
    v: Domain
    lmin: int
    L: int
    r: int                      # time DG degree
    dt: float
    delta: float                # streamline-diffusion parameter
    nstrips: int
    # beta[c] for c in 0..2d-1: None or (scale, x_field_names, v_field_names)
    beta: list
    # sigma: list of (scale, x_field_names, v_field_names)
    sigma: list
    xfields: dict               # name -> callable(coords (n,d)) -> (n,)
    vfields: dict
    u0: Optional[Callable] = None       # u0(X, V) with broadcasting
    f: Optional[Callable] = None        # f(t, X, V)
    g: Optional[Callable] = None        # g(t, X, V) (only its inflow trace matters)
    exact: Optional[Callable] = None    # exact solution u(t, X, V) if known
    seed: int = 0
    noise: float = 0.0                  # amplitude of N(0,1) noise on u0 coefficients
    # coefficients that depend on time: t -> (xfields, vfields) at time t, the same
    # names as xfields / vfields (which then give the fields' layout only)
    tfields: Optional[Callable] = None
    tquad: int = 0                      # time quadrature points per strip (0: r + 2)

    @property
    def d(self):
        return self.x.d

    @property
    def R(self):
        return self.r + 1


def lattice_shape(dom: Domain, level: int):
    m = 2 ** level if dom.periodic else 2 ** level + 1
    return (m,) * dom.d


def lattice_coords(dom: Domain, level: int) -> np.ndarray:
    """Node coordinates of the level-`level` lattice, shape (n, d), C order."""
    shape = lattice_shape(dom, level)
    idx = np.indices(shape).reshape(dom.d, -1).T.astype(np.float64)
    lo = np.asarray(dom.lo, float)
    hi = np.asarray(dom.hi, float)
    return lo + idx * ((hi - lo) / 2 ** level)


def nodal_fields(w: Workload):
    """Sample every named field at the finest-level nodes of its domain."""
    X = lattice_coords(w.x, w.L)
    V = lattice_coords(w.v, w.L)
    fx = {k: np.ascontiguousarray(fn(X), dtype=np.float64) for k, fn in w.xfields.items()}
    fv = {k: np.ascontiguousarray(fn(V), dtype=np.float64) for k, fn in w.vfields.items()}
    return fx, fv


def grid_levels(w: Workload):
    """Upper-diagonal and lower-diagonal component grids as (lx, lv) pairs.

    Upper: lx + lv = L + lmin, ordered by increasing lx.  Lower (the
    combination-technique diagonal): lx + lv = L + lmin - 1.
    """
    s = w.L + w.lmin
    upper = [(lx, s - lx) for lx in range(w.lmin, w.L + 1)]
    lower = [(lx, s - 1 - lx) for lx in range(w.lmin, w.L)]
    return upper, lower


def gauss_legendre_times(t0: float, dt: float, nq: int):
    """Gauss-Legendre nodes and weights on [t0, t0+dt]."""
    xg, wg = np.polynomial.legendre.leggauss(nq)
    return t0 + 0.5 * dt * (xg + 1.0), 0.5 * dt * wg


def sample_on_grids(w: Workload, grids, fn, t=None) -> np.ndarray:
    """Values of fn at the nodes of each component grid (x, v), concatenated.

    fn(X, V) (or fn(t, X, V) when t is given) with X, V broadcast arrays whose
    last axis is the coordinate; each grid block is [n_x][n_v], v fastest.
    """
    out = []
    for lx, lv in grids:
        X = lattice_coords(w.x, lx)[:, None, :]
        V = lattice_coords(w.v, lv)[None, :, :]
        val = fn(X, V) if t is None else fn(t, X, V)
        out.append(np.broadcast_to(val, (X.shape[0], V.shape[1])).ravel())
    return np.concatenate(out) if out else np.zeros(0)


def random_vector(n: int, seed: int, batch: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch, n))


def h_min(x: Domain, v: Domain, L: int) -> float:
    hx = min((b - a) for a, b in zip(x.lo, x.hi)) / 2 ** L
    hv = min((b - a) for a, b in zip(v.lo, v.hi)) / 2 ** L
    return min(hx, hv)


def _coord(i):
    return lambda P: P[:, i].copy()


def _ones(P):
    return np.ones(P.shape[0])


# ----------------------------------------------------------------------------
# The five benchmark workloads and the paper's first experiment.
# ----------------------------------------------------------------------------

def config_c1(seed: int = 0) -> Workload:
    """2D phase space (d=1), FP64, exact solution sin(2pi(x-vt)) exp(-4v^2)."""
    x = Domain(1, (0.0,), (1.0,))
    v = Domain(1, (-1.0,), (1.0,))
    L = 6

    def exact(t, X, V):
        x, vv = X[..., 0], V[..., 0]
        return np.sin(2 * np.pi * (x - vv * t)) * np.exp(-4 * vv ** 2)

    return Workload(
        name="c1_d1_r0_L6", x=x, v=v, lmin=1, L=L, r=0, dt=1.0 / 64,
        delta=0.5 * h_min(x, v, L), nstrips=8,
        beta=[(1.0, (), ("v0",)), None], sigma=[],
        xfields={}, vfields={"v0": _coord(0)},
        u0=lambda X, V: exact(0.0, X, V), f=None, g=exact, exact=exact,
        seed=seed, noise=1e-3)


def _bump2(t, X, V):
    # X, V: (..., 2) broadcast arrays
    s = X - V * t - 0.5
    return np.exp(-20 * np.sum(s * s, axis=-1) - 4 * np.sum(V * V, axis=-1))


def config_c2(seed: int = 0, L: int = 7) -> Workload:
    """4D phase space (d=2), r=1, sigma(v)=0.1|v|^2, Gaussian-bump exact solution."""
    x = Domain(2, (0.0, 0.0), (1.0, 1.0))
    v = Domain(2, (-1.0, -1.0), (1.0, 1.0))

    def exact(t, X, V):
        return _bump2(t, X, V)

    def forcing(t, X, V):      # f = sigma*u, since u solves the sigma-free transport
        return 0.1 * np.sum(V * V, axis=-1) * _bump2(t, X, V)

    return Workload(
        name=f"c2_d2_r1_L{L}", x=x, v=v, lmin=0, L=L, r=1, dt=1.0 / 64,
        delta=0.5 * h_min(x, v, L), nstrips=4,
        beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), None, None],
        sigma=[(0.1, (), ("v0", "v0")), (0.1, (), ("v1", "v1"))],
        xfields={}, vfields={"v0": _coord(0), "v1": _coord(1)},
        u0=lambda X, V: exact(0.0, X, V), f=forcing, g=exact, exact=exact, seed=seed)


def config_c3(seed: int = 0, L: int = 6) -> Workload:
    """6D phase space (d=3), r=0, beta=(v, 0): operator-apply throughput."""
    x = Domain(3, (0.0,) * 3, (1.0,) * 3)
    v = Domain(3, (-1.0,) * 3, (1.0,) * 3)
    return Workload(
        name=f"c3_d3_r0_L{L}", x=x, v=v, lmin=0, L=L, r=0, dt=1.0 / 64,
        delta=0.5 * h_min(x, v, L), nstrips=1,
        beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), (1.0, (), ("v2",)), None, None, None],
        sigma=[], xfields={}, vfields={f"v{i}": _coord(i) for i in range(3)}, seed=seed)


def config_c4_member(i: int, seed: int = 0, L: Optional[int] = None, tvary: float = 0.0) -> Workload:
    """One of the 64 batched 4D problems: beta=(v, a_i), sigma_i, Fourier forcing.
    L overrides the drawn level (smaller members for parity tests).  tvary > 0 makes
    the coefficients depend on time: a_i + tvary b_i t and sigma_i (1 + tvary sin(2 pi t)),
    b_i ~ U[-1, 1]^2 (drawn after everything else, so the other draws are unchanged)."""
    rng = np.random.default_rng([seed, i])
    L_drawn = int(rng.integers(5, 8))
    L = L_drawn if L is None else int(L)
    a = rng.uniform(-1.0, 1.0, size=2)
    sig = float(rng.uniform(0.0, 0.5))
    modes = []
    for _ in range(8):
        while True:
            k = rng.integers(-2, 3, size=4)
            if np.any(k != 0):
                break
        amp = rng.standard_normal() / float(np.sum(k * k))
        th = rng.uniform(0, 2 * np.pi)
        modes.append((k.astype(float), amp, th))
    x = Domain(2, (0.0, 0.0), (1.0, 1.0))
    v = Domain(2, (-1.0, -1.0), (1.0, 1.0))

    def forcing(t, X, V):
        out = 0.0
        for k, amp, th in modes:
            out = out + amp * np.cos(2 * np.pi * (X @ k[:2]) + np.pi * (V @ k[2:]) + th)
        return out

    if tvary <= 0.0:
        return Workload(
            name=f"c4_member{i}_L{L}", x=x, v=v, lmin=0, L=L, r=1, dt=1.0 / 64,
            delta=0.5 * h_min(x, v, L), nstrips=4,
            beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), (float(a[0]), (), ()), (float(a[1]), (), ())],
            sigma=[(sig, (), ())], xfields={}, vfields={"v0": _coord(0), "v1": _coord(1)},
            u0=None, f=forcing, g=None, seed=seed)
    b = rng.uniform(-1.0, 1.0, size=2)

    def consts(t):
        vals = {"a0": a[0] + tvary * b[0] * t, "a1": a[1] + tvary * b[1] * t,
                "s": sig * (1.0 + tvary * np.sin(2 * np.pi * t))}
        return {k: (lambda P, c=c: np.full(len(P), c)) for k, c in vals.items()}

    vf = {"v0": _coord(0), "v1": _coord(1)}
    return Workload(
        name=f"c4_member{i}_L{L}_t", x=x, v=v, lmin=0, L=L, r=1, dt=1.0 / 64,
        delta=0.5 * h_min(x, v, L), nstrips=4,
        beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), (1.0, ("a0",), ()), (1.0, ("a1",), ())],
        sigma=[(1.0, ("s",), ())], xfields=consts(0.0), vfields=vf,
        u0=None, f=forcing, g=None, seed=seed, tfields=lambda t: (consts(t), dict(vf)))


def config_c4(seed: int = 0, n: int = 64):
    return [config_c4_member(i, seed) for i in range(n)]


def config_c5(seed: int = 0, L: int = 7) -> Workload:
    """4D Vlasov-type transport step with a frozen random periodic field E(x)."""
    rng = np.random.default_rng(seed)
    ks = []
    for k1 in range(0, 6):
        for k2 in range(-5, 6):
            if k1 > 0 or (k1 == 0 and k2 > 0):
                ks.append((k1 * k1 + k2 * k2, k1, k2))
    ks.sort()
    ks = [(k1, k2) for _, k1, k2 in ks[:16]]
    th = rng.uniform(0, 2 * np.pi, size=len(ks))

    def efield(comp):
        def fn(P):
            out = np.zeros(P.shape[0])
            for (k1, k2), t in zip(ks, th):
                kk = k1 * k1 + k2 * k2
                kc = (k1, k2)[comp]
                out += (0.05 / kk) * 2 * np.pi * kc * np.sin(2 * np.pi * (k1 * P[:, 0] + k2 * P[:, 1]) + t)
            return out
        return fn

    x = Domain(2, (0.0, 0.0), (1.0, 1.0), periodic=True)
    v = Domain(2, (-6.0, -6.0), (6.0, 6.0))

    def u0(X, V):
        return (1 + 0.01 * np.cos(2 * np.pi * X[..., 0])) * np.exp(-0.5 * np.sum(V * V, axis=-1)) / (2 * np.pi)

    return Workload(
        name=f"c5_d2_r0_L{L}", x=x, v=v, lmin=0, L=L, r=0, dt=1.0 / 64,
        delta=0.5 * h_min(x, v, L), nstrips=32,
        beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), (1.0, ("E0",), ()), (1.0, ("E1",), ())],
        sigma=[], xfields={"E0": efield(0), "E1": efield(1)},
        vfields={"v0": _coord(0), "v1": _coord(1)}, u0=u0, seed=seed)


def config_table1(Lp: int, r: int = 1, d: int = 1) -> Workload:
    """Sect. 5.1: periodic advection with beta = 1 in all 2d directions on [0,1]^(2d),
    u0 = sin(2 pi sum_i (x_i + v_i)), one period T = 1/(2d).

    Paper level Lp (4 cells per axis at paper level 1) maps to lmin=2, L=Lp+1; delta is
    the finest edge length; 2**(Lp+1) time steps.
    """
    x = Domain(d, (0.0,) * d, (1.0,) * d, periodic=True)
    v = Domain(d, (0.0,) * d, (1.0,) * d, periodic=True)
    nst = 2 ** (Lp + 1)

    def exact(t, X, V):
        return np.sin(2 * np.pi * (X.sum(axis=-1) + V.sum(axis=-1) - 2 * d * t))

    return Workload(
        name=f"table1_d{d}_Lp{Lp}", x=x, v=v, lmin=2, L=Lp + 1, r=r, dt=1.0 / (2 * d) / nst,
        delta=2.0 ** (-(Lp + 1)), nstrips=nst,
        beta=[(1.0, (), ())] * (2 * d), sigma=[], xfields={}, vfields={},
        u0=lambda X, V: exact(0.0, X, V), f=None, g=None, exact=exact)


def _vp_workload(name, d, paper_level, r, dt, length, vmax, f0, E, tend):
    """Periodic (0, length)^d x (-vmax, vmax)^d for the Vlasov-Poisson runs of Sect. 5.3,
    four cells per axis on the coarsest level (lmin = 2, so the paper's level L is
    L + 1 here), beta = (v, -E(x)) with E the nodal field on the finest x-lattice,
    [d][n] (zero when None), delta = 0.5 h_min, strips up to time tend."""
    lmin = 2
    L = lmin + paper_level - 1
    x = Domain(d, (0.0,) * d, (length,) * d, periodic=True)
    v = Domain(d, (-vmax,) * d, (vmax,) * d)
    nfine = (2 ** L) ** d
    Ef = np.zeros((d, nfine)) if E is None else np.asarray(E, float).reshape(d, nfine)
    beta = [(1.0, (), (f"v{i}",)) for i in range(d)] + [(-1.0, (f"E{i}",), ()) for i in range(d)]
    h = min(length, 2 * vmax) / 2 ** L
    return Workload(
        name=f"{name}_d{d}_L{paper_level}", x=x, v=v, lmin=lmin, L=L, r=r, dt=dt, delta=0.5 * h,
        nstrips=int(round(tend / dt)), beta=beta, sigma=[],
        xfields={f"E{i}": (lambda P, i=i: Ef[i].copy()) for i in range(d)},
        vfields={f"v{i}": _coord(i) for i in range(d)},
        u0=f0, f=None, g=None, exact=None)


def config_landau(d: int = 1, paper_level: int = 5, r: int = 1, dt: float = 0.5, alpha: float = 1e-2,
                  k: float = 0.5, E=None, vmax: float = 6.0) -> Workload:
    """Landau damping (Sect. 5.3): periodic (0, 4 pi)^d x (-vmax, vmax)^d,
    f0 = exp(-|v|^2/2) / (2 pi)^(d/2) * (1 + alpha sum_i cos(k x_i)), on [0, 50]."""

    def f0(X, V):
        return (np.exp(-0.5 * np.sum(V * V, axis=-1)) / (2 * np.pi) ** (d / 2)
                * (1 + alpha * np.sum(np.cos(k * X), axis=-1)))

    return _vp_workload("landau", d, paper_level, r, dt, 4 * np.pi, vmax, f0, E, 50.0)


def config_twostream(d: int = 1, paper_level: int = 5, r: int = 1, dt: float = 0.5, alpha: float = 1e-3,
                     k: float = 0.2, v0: float = 2.4, vmax: float = 9.0, E=None) -> Workload:
    """Two-stream instability (Sect. 5.3): periodic (0, 10 pi)^d x (-9, 9)^d,
    f0 = prod_i (exp(-(v_i - v0)^2/2) + exp(-(v_i + v0)^2/2)) / (2 sqrt(2 pi))^d
         * (1 + alpha sum_i cos(k x_i)), on [0, 50] (the Landau runs' interval and strips)."""

    def f0(X, V):
        beams = np.prod(np.exp(-0.5 * (V - v0) ** 2) + np.exp(-0.5 * (V + v0) ** 2), axis=-1)
        return beams / (2 * np.sqrt(2 * np.pi)) ** d * (1 + alpha * np.sum(np.cos(k * X), axis=-1))

    return _vp_workload("twostream", d, paper_level, r, dt, 2 * np.pi / k, vmax, f0, E, 50.0)


def with_time_fields(w: Workload, tfields, tquad: int = 0) -> Workload:
    """The workload with coefficients given as functions of time (tfields: t -> fields)."""
    w.tfields = tfields
    w.tquad = tquad
    return w


def config_timedep_exact(d: int, r: int, L: int) -> Workload:
    """u = p(x, v) + q t affine in space with beta_v moving in time: beta = (v, c0 + c1 x + c2 t)
    (d = 1) or (v, a + b t) (d = 2); f = d_t u + beta.grad u + sigma u and g = u lie in the
    discrete space, so every strip reproduces u (consistency and uniqueness, as for
    constant coefficients), provided the time quadrature integrates the degree-4
    integrands exactly (r + 2 Gauss points)."""
    sig = 0.3
    qt = 0.7 if r >= 1 else 0.0
    if d == 1:
        x = Domain(1, (0.0,), (1.0,))
        v = Domain(1, (-1.0,), (1.0,))
        c0, c1, c2 = 0.5, 0.8, 0.9

        def u(t, X, V):
            return 1.0 + 0.6 * X[..., 0] - 0.9 * V[..., 0] + qt * t

        def f(t, X, V):
            return qt + 0.6 * V[..., 0] + (c0 + c1 * X[..., 0] + c2 * t) * (-0.9) + sig * u(t, X, V)

        def tf(t):
            return {"c": lambda P, t=t: c0 + c1 * P[:, 0] + c2 * t}, {"v0": lambda P: P[:, 0].copy()}

        w = Workload(name="exact_t_d1", x=x, v=v, lmin=1, L=L, r=r, dt=0.05, delta=0.04, nstrips=2,
                     beta=[(1.0, (), ("v0",)), (1.0, ("c",), ())], sigma=[(sig, (), ())],
                     xfields={"c": lambda P: c0 + c1 * P[:, 0]}, vfields={"v0": lambda P: P[:, 0].copy()},
                     u0=lambda X, V: u(0.0, X, V), f=f, g=u, exact=u)
        return with_time_fields(w, tf)
    x = Domain(2, (0.0, 0.0), (1.0, 1.0))
    v = Domain(2, (-1.0, -1.0), (1.0, 1.0))
    a = np.array([0.5, -0.3])
    bt = np.array([0.6, 0.4])
    bx = np.array([0.4, -0.7])
    cv = np.array([0.2, 0.5])

    def u(t, X, V):
        return 1.0 + X @ bx + V @ cv + qt * t

    def f(t, X, V):
        return qt + V @ bx + float(cv @ (a + bt * t)) + sig * u(t, X, V)

    def tf(t):
        return ({"a0": lambda P, t=t: np.full(len(P), a[0] + bt[0] * t),
                 "a1": lambda P, t=t: np.full(len(P), a[1] + bt[1] * t)},
                {"v0": lambda P: P[:, 0].copy(), "v1": lambda P: P[:, 1].copy()})

    w = Workload(name="exact_t_d2", x=x, v=v, lmin=0, L=L, r=r, dt=0.05, delta=0.05, nstrips=2,
                 beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), (1.0, ("a0",), ()), (1.0, ("a1",), ())],
                 sigma=[(sig, (), ())],
                 xfields={"a0": lambda P: np.full(len(P), a[0]), "a1": lambda P: np.full(len(P), a[1])},
                 vfields={"v0": lambda P: P[:, 0].copy(), "v1": lambda P: P[:, 1].copy()},
                 u0=lambda X, V: u(0.0, X, V), f=f, g=u, exact=u)
    return with_time_fields(w, tf)


def config_tiny(kind: str) -> Workload:
    """Small problems exercising every term of the operator (used for brute-force checks)."""
    if kind == "d1":
        x = Domain(1, (0.0,), (1.0,))
        v = Domain(1, (-1.0,), (1.0,))
        return Workload(
            name="tiny_d1", x=x, v=v, lmin=1, L=3, r=1, dt=0.1, delta=0.05, nstrips=2,
            beta=[(1.0, (), ("v0",)), (0.7, ("c",), ())],
            sigma=[(0.3, ("x0",), ("v0", "v0")), (0.2, (), ())],
            xfields={"x0": _coord(0), "c": lambda P: 0.5 + P[:, 0] ** 2},
            vfields={"v0": _coord(0)},
            u0=lambda X, V: np.cos(np.pi * X[..., 0]) * (1 - V[..., 0] ** 2),
            f=lambda t, X, V: np.sin(X[..., 0] + V[..., 0] + t),
            g=lambda t, X, V: 1 + X[..., 0] * V[..., 0] + t,
            exact=None)
    if kind == "d1p":
        x = Domain(1, (0.0,), (2.0,), periodic=True)
        v = Domain(1, (-1.0,), (1.0,))
        return Workload(
            name="tiny_d1p", x=x, v=v, lmin=1, L=3, r=0, dt=0.1, delta=0.05, nstrips=2,
            beta=[(1.0, (), ("v0",)), (-0.4, ("s",), ())], sigma=[],
            xfields={"s": lambda P: np.sin(np.pi * P[:, 0])}, vfields={"v0": _coord(0)},
            u0=lambda X, V: np.exp(-V[..., 0] ** 2) * (1 + 0.5 * np.cos(np.pi * X[..., 0])),
            exact=None)
    if kind == "d2":
        x = Domain(2, (0.0, 0.0), (1.0, 1.0))
        v = Domain(2, (-1.0, -1.0), (1.0, 1.0))
        return Workload(
            name="tiny_d2", x=x, v=v, lmin=0, L=2, r=1, dt=0.05, delta=0.1, nstrips=2,
            beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), (0.5, (), ()), (-0.3, ("x0",), ())],
            sigma=[(0.1, (), ("v0", "v0")), (0.1, (), ("v1", "v1"))],
            xfields={"x0": _coord(0)}, vfields={"v0": _coord(0), "v1": _coord(1)},
            u0=lambda X, V: _bump2(0.0, X, V), f=lambda t, X, V: 0.1 * _bump2(t, X, V),
            g=_bump2, exact=None)
    if kind == "d3":
        x = Domain(3, (0.0,) * 3, (1.0,) * 3)
        v = Domain(3, (-1.0,) * 3, (1.0,) * 3)
        return Workload(
            name="tiny_d3", x=x, v=v, lmin=0, L=1, r=0, dt=0.05, delta=0.1, nstrips=1,
            beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), (1.0, (), ("v2",)), (0.2, (), ()), None, None],
            sigma=[(0.05, (), ())], xfields={}, vfields={f"v{i}": _coord(i) for i in range(3)},
            exact=None)
    raise ValueError(kind)
