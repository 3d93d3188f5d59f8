"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a transposed factor, a wrong level) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import (Domain, Workload, config_c1, config_table1, config_tiny, config_timedep_exact,
                       grid_levels, lattice_coords, with_time_fields)
from oracle.brute import Brute
from oracle.ct import CTPreconditioner
from oracle.fe import assemble
from oracle.krylov import fgmres
from oracle.mesh import Lattice, embedding
from oracle.operator import Problem
from oracle import strip
from oracle.timedg import time_matrices

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.strip() and not line.startswith("#"):
            rows.append(line.split())
    return rows


# --- T1: Table 1 dof column ---------------------------------------------------------

def test_table1_dof_column_counts():
    """dim V_L = sum over upper n_x n_v - sum over lower n_x n_v reproduces all 31 entries."""
    for d, r, Lp, dof in _read("table1_dof.txt"):
        d, r, Lp, dof = int(d), int(r), int(Lp), int(dof)
        # periodic, 4 cells at paper level 1; order-r elements have r*cells nodes per axis
        n = lambda lp: (r * 4 * 2 ** (lp - 1)) ** d
        up = sum(n(l1) * n(Lp + 1 - l1) for l1 in range(1, Lp + 1))
        lo = sum(n(l1) * n(Lp - l1) for l1 in range(1, Lp))
        assert up - lo == dof, (d, r, Lp)


@pytest.mark.parametrize("d,Lp", [(1, 1), (1, 2), (1, 3), (1, 4), (2, 1), (2, 2)])
def test_table1_dof_equals_rank_of_spanning_set(d, Lp):
    """The rank of the sparse-grid mass matrix (Gram matrix of the spanning set) is dim V_L."""
    x = Domain(d, (0.0,) * d, (1.0,) * d, periodic=True)
    w = Workload(name="t", x=x, v=x, lmin=2, L=Lp + 1, r=0, dt=1.0, delta=0.0, nstrips=1,
                 beta=[None] * (2 * d), sigma=[], xfields={}, vfields={})
    P = Problem(w)
    M = P.assembled(P.mass_terms()).toarray()
    rank = np.linalg.matrix_rank(M, tol=1e-10 * np.abs(M).max())
    expect = {int(a[2]): int(a[3]) for a in _read("table1_dof.txt") if int(a[0]) == d and int(a[1]) == 1}
    assert rank == expect[Lp]


# --- T2/T3: factor matrices ---------------------------------------------------------

def test_1d_closed_forms():
    lat = Lattice(1, (0.0,), (2.0,), 4)
    h = 2.0 / 16
    xs = lattice_coords(Domain(1, (0.0,), (2.0,)), 4)[:, 0]
    M = assemble(lat, "mass", []).toarray()
    D = assemble(lat, "deriv", [], a=0).toarray()
    S = assemble(lat, "stiff", [], a=0, b=0).toarray()
    Mv = assemble(lat, "mass", [xs]).toarray()
    k = 7
    assert np.allclose(M[k, k - 1:k + 2], h * np.array([1 / 6, 2 / 3, 1 / 6]), atol=1e-15)
    assert np.allclose(D[k, k - 1:k + 2], [-0.5, 0.0, 0.5], atol=1e-15)
    assert np.allclose(S[k, k - 1:k + 2], np.array([-1.0, 2.0, -1.0]) / h, atol=1e-12)
    assert math.isclose(Mv[k, k], 2 * h * xs[k] / 3, rel_tol=1e-13)
    assert math.isclose(Mv[k, k + 1], h * (xs[k] + xs[k + 1]) / 12, rel_tol=1e-13)
    # boundary rows: half mass, one-sided derivative
    assert np.allclose(M[0, :2], h * np.array([1 / 3, 1 / 6]))
    assert np.allclose(D[0, :2], [-0.5, 0.5])


@pytest.mark.parametrize("d", [1, 2, 3])
def test_factor_identities(d):
    lo, hi = (-1.0,) * d, (1.0,) * d
    fine = Lattice(d, lo, hi, 2)
    coarse = Lattice(d, lo, hi, 1)
    one = np.ones(fine.n)
    M = assemble(fine, "mass", [])
    assert math.isclose(one @ M @ one, 2.0 ** d, rel_tol=1e-13)
    for a in range(d):
        assert np.abs(assemble(fine, "deriv", [], a=a) @ one).max() < 1e-13
        for b in range(d):
            S = assemble(fine, "stiff", [], a=a, b=b)
            assert np.abs(S @ one).max() < 1e-12
            assert np.abs((S.T - assemble(fine, "stiff", [], a=b, b=a))).max() < 1e-13
    E = embedding(coarse, fine)
    assert np.allclose(E @ np.ones(coarse.n), 1.0)
    # Galerkin identity E^T X_fine E = X_coarse for polynomial weights (Sect. 4.2)
    Xf = lattice_coords(Domain(d, lo, hi), 2)
    Xc = lattice_coords(Domain(d, lo, hi), 1)
    for kind, kw in (("mass", {}), ("deriv", {"a": d - 1}), ("stiff", {"a": 0, "b": d - 1})):
        wf = [Xf[:, 0], Xf[:, d - 1]]
        wc = [Xc[:, 0], Xc[:, d - 1]]
        lhs = (E.T @ assemble(fine, kind, wf, **kw) @ E).toarray()
        rhs = assemble(coarse, kind, wc, **kw).toarray()
        assert np.abs(lhs - rhs).max() < 1e-13
    if d > 1:
        F = assemble(fine, "face", [], face=(0, 1))
        assert math.isclose(one @ F @ one, 2.0 ** (d - 1), rel_tol=1e-13)


def test_prolongation_reproduces_linear_functions():
    dom = Domain(2, (0.0, -1.0), (1.0, 3.0))
    for l in range(0, 3):
        c = Lattice(2, dom.lo, dom.hi, l)
        f = Lattice(2, dom.lo, dom.hi, l + 1)
        Xc, Xf = c.node_coords(), f.node_coords()
        lin = lambda X: 0.3 + 2 * X[:, 0] - 0.7 * X[:, 1]
        assert np.allclose(embedding(c, f) @ lin(Xc), lin(Xf), atol=1e-13)


# --- time-DG blocks ------------------------------------------------------------------

def test_time_matrices_closed_forms():
    dt = 0.3
    Mt, Tt, Ct, Gt = time_matrices(0, dt)
    assert np.allclose(Mt, [[dt]]) and np.allclose(Tt, 0) and np.allclose(Ct, 0) and np.allclose(Gt, 1)
    Mt, Tt, Ct, Gt = time_matrices(1, dt)
    assert np.allclose(Mt, np.diag([dt, dt / 3]))
    assert np.allclose(Tt, [[0, 2], [0, 0]])
    assert np.allclose(Ct, [[0, 0], [0, 4 / dt]])
    assert np.allclose(Gt, [[1, -1], [-1, 1]])


@pytest.mark.parametrize("r", [0, 1])
def test_pade_reaction_step(r):
    """beta=0, delta=0, sigma=c: each strip maps U to R(c dt) U with the (r, r+1) Pade
    approximant of exp(-z) -- the classical DG(r) time-stepping property."""
    sig, dt = 0.7, 0.25
    x = Domain(1, (0.0,), (1.0,))
    v = Domain(1, (-1.0,), (1.0,))
    w = Workload(name="pade", x=x, v=v, lmin=1, L=3, r=r, dt=dt, delta=0.0, nstrips=2,
                 beta=[None, None], sigma=[(sig, (), ())], xfields={}, vfields={},
                 u0=lambda X, V: np.cos(3 * X[..., 0]) + V[..., 0] ** 2)
    P = Problem(w)
    sols, st = strip.march(P, tol=1e-13)
    z = sig * dt
    Rz = 1 / (1 + z) if r == 0 else (1 - z / 3) / (1 + 2 * z / 3 + z * z / 6)
    prev = strip.initial_coefficients(P)
    for u in sols:
        tr = strip.trace_right(P, u, P.R)
        e = tr - Rz * prev
        # squared L2 norm of the difference function (the coefficients are not unique)
        assert abs(e @ P.apply_mass(e)) < 1e-14 * (tr @ P.apply_mass(tr))
        prev = tr


# --- T4: brute force (weak form by quadrature) vs Kronecker form ---------------------

@pytest.mark.parametrize("kind", ["d1", "d1p", "d2"])
def test_brute_force_equals_kronecker(kind):
    w = config_tiny(kind)
    A2 = Problem(w).assembled().toarray()
    A1 = Brute(w).matrix()
    assert np.abs(A1 - A2).max() <= 1e-12 * np.abs(A1).max()


@pytest.mark.slow
def test_brute_force_equals_kronecker_d3():
    w = config_tiny("d3")
    A2 = Problem(w).assembled().toarray()
    A1 = Brute(w, nq_x=3, nq_v=4).matrix()
    assert np.abs(A1 - A2).max() <= 1e-12 * np.abs(A1).max()


def test_blockwise_order_equals_assembled():
    for kind in ("d1", "d2"):
        P = Problem(config_tiny(kind))
        u = np.random.default_rng(1).standard_normal(P.ndof)
        assert np.abs(P.apply(u) - P.assembled() @ u).max() < 1e-13


# --- T6/T7/T8: properties of the full operator ----------------------------------------

@pytest.mark.parametrize("kind", ["d1", "d2"])
def test_kernel_vectors(kind):
    """+E c on one upper grid and -E' c on its neighbour represent the zero function."""
    P = Problem(config_tiny(kind))
    rng = np.random.default_rng(2)
    for i in range(len(P.upper) - 1):
        (lx, lv), (lx2, lv2) = P.upper[i], P.upper[i + 1]
        low = (lx, lv - 1)
        c = rng.standard_normal((P.R, P.nx(low[0]), P.nv(low[1])))
        z = [np.zeros((P.R, P.nx(a), P.nv(b))) for a, b in P.upper]
        Ev = P.E("v", lv, lv - 1)
        Ex = P.E("x", lx2, lx)
        z[i] = np.stack([(Ev @ cs.T).T for cs in c])
        z[i + 1] = -np.stack([Ex @ cs for cs in c])
        z = np.concatenate([a.ravel() for a in z])
        Az = P.apply(z)
        assert np.abs(Az).max() < 1e-13 * max(1.0, np.abs(P.apply(np.abs(z))).max())


def test_constants_consistency():
    for kind in ("d1", "d2"):
        P = Problem(config_tiny(kind))
        u = np.random.default_rng(3).standard_normal(P.ndof)
        blocks = P.split(P.apply(u))
        sums = np.array([b.reshape(P.R, -1).sum(axis=1) for b in blocks])
        assert np.abs(sums - sums[0]).max() < 1e-12 * np.abs(sums).max()


@pytest.mark.parametrize("w", [config_table1(2), config_tiny("d1"), config_tiny("d1p")],
                         ids=["table1", "tiny_d1", "tiny_d1p"])
def test_symmetric_part_psd(w):
    """Lemma 1: A(v,v) >= 1/2 |||v|||^2 >= 0, so (A + A^T)/2 is positive semi-definite."""
    A = Problem(w).assembled().toarray()
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > -1e-12 * np.abs(ev).max()


# --- T9: mass balance -------------------------------------------------------------------

def test_mass_conservation_periodic_x():
    """sigma=0, f=0, x periodic and beta_v=0: (U_j^-, 1) is conserved strip by strip."""
    x = Domain(1, (0.0,), (1.0,), periodic=True)
    v = Domain(1, (-1.0,), (1.0,))
    w = Workload(name="mass", x=x, v=v, lmin=1, L=4, r=1, dt=0.05, delta=0.03, nstrips=3,
                 beta=[(1.0, (), ("v0",)), None], sigma=[], xfields={},
                 vfields={"v0": lambda P: P[:, 0].copy()},
                 u0=lambda X, V: (1 + np.sin(2 * np.pi * X[..., 0])) * np.exp(-3 * V[..., 0] ** 2))
    P = Problem(w)
    sols, _ = strip.march(P, tol=1e-13)
    n0 = P.nx(P.upper[0][0]) * P.nv(P.upper[0][1])

    def mass(u1):
        return P.apply_mass(u1)[:n0].sum()

    m0 = mass(strip.initial_coefficients(P))
    for u in sols:
        assert abs(mass(strip.trace_right(P, u, P.R)) - m0) < 1e-11 * abs(m0)


def test_mass_decay_with_reaction():
    """sigma const, beta=(v, 0) periodic in x: d/dt (U,1) = -sigma (U,1) holds weakly:
    (U_j^-,1) - (U_{j-1}^-,1) = -sigma int_{I_j} (U,1) dt."""
    sig = 0.4
    x = Domain(1, (0.0,), (1.0,), periodic=True)
    v = Domain(1, (-1.0,), (1.0,))
    w = Workload(name="mass2", x=x, v=v, lmin=1, L=4, r=1, dt=0.1, delta=0.02, nstrips=2,
                 beta=[(1.0, (), ("v0",)), None], sigma=[(sig, (), ())], xfields={},
                 vfields={"v0": lambda P: P[:, 0].copy()},
                 u0=lambda X, V: (1 + np.cos(2 * np.pi * X[..., 0])) * (1 - V[..., 0] ** 2))
    P = Problem(w)
    sols, _ = strip.march(P, tol=1e-13)
    n0 = P.nx(P.upper[0][0]) * P.nv(P.upper[0][1])
    mass = lambda u1: P.apply_mass(u1)[:n0].sum()
    prev = mass(strip.initial_coefficients(P))
    for u in sols:
        blk = P.split(u)
        # int_{I_j} (U,1) dt = dt * (U_0 coefficient, 1) since int eta_1 = 0
        u0part = np.concatenate([b[0].ravel() for b in blk])
        integral = w.dt * mass(u0part)
        now = mass(strip.trace_right(P, u, P.R))
        assert abs((now - prev) + sig * integral) < 1e-11
        prev = now


# --- T12 and Krylov -------------------------------------------------------------------------

def test_ct_single_grid_is_exact_inverse():
    w = config_tiny("d1")
    w.L = w.lmin                      # one upper grid, no lower grid
    P = Problem(w)
    b = np.random.default_rng(4).standard_normal(P.ndof)
    x, st = fgmres(P.apply, b, CTPreconditioner(P), tol=1e-12)
    assert st["iters"] == 1 and st["rel"] < 1e-12


def test_ct_linear_and_interpolation_exact():
    P = Problem(config_tiny("d2"))
    ct = CTPreconditioner(P)
    rng = np.random.default_rng(5)
    r1, r2 = rng.standard_normal(P.ndof), rng.standard_normal(P.ndof)
    assert np.abs(ct(2 * r1 - 3 * r2) - (2 * ct(r1) - 3 * ct(r2))).max() < 1e-10
    # the combination formula reproduces any function of V_L: take a hat product on grid (1,1)
    g = P.upper[1]
    Xc = lattice_coords(P.w.x, g[0])
    Vc = lattice_coords(P.w.v, g[1])
    kx, kv = 4, 3
    latx = Lattice(2, P.w.x.lo, P.w.x.hi, g[0])
    latv = Lattice(2, P.w.v.lo, P.w.v.hi, g[1])

    def hat(X, V):
        sh = X.shape[:-1]
        Xf = np.broadcast_to(X, np.broadcast_shapes(X.shape, V.shape[:-1] + (2,))).reshape(-1, 2)
        Vf = np.broadcast_to(V, np.broadcast_shapes(V.shape, X.shape[:-1] + (2,))).reshape(-1, 2)
        a = latx.eval(Xf)[0][:, kx].toarray().ravel()
        b = latv.eval(Vf)[0][:, kv].toarray().ravel()
        return (a * b).reshape(np.broadcast_shapes(X.shape[:-1], V.shape[:-1]))

    ui = strip.interpolate(P, hat)
    ref = np.zeros(P.ndof // P.R)
    off = sum(P.nx(a) * P.nv(b) for a, b in P.upper[:1])
    ref[off + kx * P.nv(g[1]) + kv] = 1.0
    e = ui - ref
    assert e @ P.apply_mass(e) < 1e-26


@pytest.mark.parametrize("kind", ["d1", "d1p", "d2"])
def test_ct_reproduces_functions_common_to_all_grids(kind):
    """Algorithm 1's grid problems are the operator restricted to each component
    space (the lower grids' residuals are x-restrictions of their upper
    partners', i.e. the same dual values), so for u in the space every grid
    contains, V_lmin (x) V_lmin, each grid solve returns u on that grid; the
    combination (one more upper than lower grid) returns u itself:
    P_CT(A u) = u.  A dropped or sign-flipped lower-grid term, a transposed
    restriction or a wrong grid operator breaks it."""
    P = Problem(config_tiny(kind))
    lmin, R = P.w.lmin, P.R
    g0 = next(g for g in P.upper if g[0] == lmin)
    Ev = P.E("v", g0[1], lmin)
    rng = np.random.default_rng(11)
    u = np.zeros(P.ndof)
    blocks = P.split(u)
    i0 = P.upper.index(g0)
    for s in range(R):
        c = rng.standard_normal((P.nx(lmin), P.nv(lmin)))
        blocks[i0][s] = (Ev @ c.T).T
    z = CTPreconditioner(P)(P.apply(u))
    e = z - u

    def slice_of(vec, s):
        return np.concatenate([b[s].ravel() for b in P.split(vec)])

    for s in range(R):
        es, us = slice_of(e, s), slice_of(u, s)
        assert es @ P.apply_mass(es) <= 1e-22 * (us @ P.apply_mass(us))
    assert np.abs(e).max() < 1e-10 * np.abs(u).max()


def test_fgmres_solves_nonsingular_system():
    rng = np.random.default_rng(6)
    A = np.eye(40) * 3 + rng.standard_normal((40, 40)) * 0.3
    b = rng.standard_normal(40)
    x, st = fgmres(lambda v: A @ v, b, tol=1e-13, restart=10)
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-10)


# --- T10/T11: exact solutions and the paper's convergence table ----------------------------

def test_c1_exact_solution_error_small():
    w = config_c1()
    w.noise = 0.0
    P = Problem(w)
    sols, st = strip.march(P, tol=1e-10)
    assert all(s["rel"] <= 1e-10 for s in st)
    T = w.nstrips * w.dt
    e = strip.trace_right(P, sols[-1], P.R) - strip.interpolate(P, lambda X, V: w.exact(T, X, V))
    ex = strip.interpolate(P, lambda X, V: w.exact(T, X, V))
    assert np.sqrt(e @ P.apply_mass(e)) < 0.02 * np.sqrt(ex @ P.apply_mass(ex))


def test_table1_d1_r1_convergence():
    """Table 1, d=1, r=1: SD-norm errors and orders of the periodic advection test.

    The paper compares with an order-(r+1) interpolant of u in V_{L+1}; the oracle
    compares with u itself, so values are pinned to 12% and orders to 0.05 (for the
    asymptotic levels L >= 3).  Exact digits: parity unpinned.
    """
    from oracle.norms import sd_error_periodic
    table = {int(r[0]): (float(r[2]), float(r[3])) for r in _read("table1_d1_r1_errors.txt")}
    errs = {}
    for Lp in range(1, 6):
        w = config_table1(Lp)
        P = Problem(w)
        sols, st = strip.march(P, tol=1e-12)
        assert all(s["rel"] <= 1e-12 for s in st)
        errs[Lp] = sd_error_periodic(P, None, sols, w.exact)
        assert abs(errs[Lp] / table[Lp][0] - 1) < 0.12, (Lp, errs[Lp])
    for Lp in range(3, 6):
        order = np.log2(errs[Lp - 1] / errs[Lp])
        assert abs(order - table[Lp][1]) < 0.05, (Lp, order)


# --- data functionals: a solution in the discrete space is reproduced exactly --------------

def _discrete_exact_workload(d, r, L, nstrips=2):
    """u = p(x, v) + q t + e t^2 with p affine in (x, v), beta = (v, c(x)) with c affine and
    positive (d = 1) or beta = (v, a) (d = 2), sigma constant.  Then u and the data
    f = d_t u + beta.grad u + sigma u and g = u are affine in space (P1 on the coarsest
    level, so every interpolant is exact) and of degree <= r in time.  By the consistency
    of the streamline-diffusion weak form (eq:weak_form_j) and the uniqueness of the strip
    solution (Thm 2) the discrete solution of every strip is u itself.  (A bilinear term
    such as x v would not do: beta.grad u would then hold v^2, outside the P1 spaces.)"""
    sig = 0.3
    qt = 0.7 if r >= 1 else 0.0
    et = -0.4 if r >= 2 else 0.0
    if d == 1:
        x = Domain(1, (0.0,), (1.0,))
        v = Domain(1, (-1.0,), (1.0,))
        c0, c1 = 0.5, 0.8                     # beta_v = c(x) = c0 + c1 x > 0: inflow on v = -1

        def u(t, X, V):
            xx, vv = X[..., 0], V[..., 0]
            return 1.0 + 0.6 * xx - 0.9 * vv + qt * t + et * t * t

        def f(t, X, V):
            xx, vv = X[..., 0], V[..., 0]
            return (qt + 2 * et * t) + vv * 0.6 + (c0 + c1 * xx) * (-0.9) + sig * u(t, X, V)

        return Workload(name="exact_d1", x=x, v=v, lmin=1, L=L, r=r, dt=0.05, delta=0.04, nstrips=nstrips,
                        beta=[(1.0, (), ("v0",)), (1.0, ("c",), ())], sigma=[(sig, (), ())],
                        xfields={"c": lambda P: c0 + c1 * P[:, 0]}, vfields={"v0": lambda P: P[:, 0].copy()},
                        u0=lambda X, V: u(0.0, X, V), f=f, g=u, exact=u)
    x = Domain(2, (0.0, 0.0), (1.0, 1.0))
    v = Domain(2, (-1.0, -1.0), (1.0, 1.0))
    a = np.array([0.5, -0.3])
    bx = np.array([0.4, -0.7])
    cv = np.array([0.2, 0.5])

    def u(t, X, V):
        return 1.0 + X @ bx + V @ cv + qt * t + et * t * t

    def f(t, X, V):
        return (qt + 2 * et * t) + V @ bx + float(cv @ a) + sig * u(t, X, V)

    return Workload(name="exact_d2", x=x, v=v, lmin=0, L=L, r=r, dt=0.05, delta=0.05, nstrips=nstrips,
                    beta=[(1.0, (), ("v0",)), (1.0, (), ("v1",)), (float(a[0]), (), ()), (float(a[1]), (), ())],
                    sigma=[(sig, (), ())], xfields={},
                    vfields={"v0": lambda P: P[:, 0].copy(), "v1": lambda P: P[:, 1].copy()},
                    u0=lambda X, V: u(0.0, X, V), f=f, g=u, exact=u)


def _legendre_slices(P, fn, t0, dt, R):
    """Spanning coefficients of the time slices of fn on [t0, t0 + dt] for fn of degree < R in t:
    values at R distinct times, then the Legendre-Vandermonde system (no quadrature)."""
    tau = np.cos(np.pi * (np.arange(R) + 0.5) / R)
    Vd = np.polynomial.legendre.legvander(tau, R - 1)            # (R times, R slices)
    Vinv = np.linalg.inv(Vd)
    vals = [strip.interpolate(P, lambda X, V, t=t0 + 0.5 * dt * (tk + 1): fn(t, X, V)) for tk in tau]
    slices = [sum(Vinv[s, k] * vals[k] for k in range(R)) for s in range(R)]
    return slices


@pytest.mark.parametrize("d,r,L", [(1, 0, 4), (1, 1, 4), (1, 2, 3), (2, 1, 2)])
def test_discrete_exact_solution_is_reproduced(d, r, L):
    """Pins the data functionals b_f (including delta (d_t w + d_beta w)), b_g, the time
    projection of the data and the jump term: every strip must return u to rounding."""
    w = _discrete_exact_workload(d, r, L)
    P = Problem(w)
    sols, st = strip.march(P, tol=1e-13, maxit=200)
    assert all(s["rel"] <= 1e-12 for s in st)
    for j, U in enumerate(sols, start=1):
        ref = _legendre_slices(P, w.exact, (j - 1) * w.dt, w.dt, P.R)
        blocks = P.split(U)
        err2 = ref2 = 0.0
        for s in range(P.R):
            us = np.concatenate([b[s].ravel() for b in blocks])
            e = us - ref[s]
            err2 += abs(e @ P.apply_mass(e))
            ref2 += abs(ref[s] @ P.apply_mass(ref[s]))
        assert np.sqrt(err2 / ref2) < 1e-10, (j, np.sqrt(err2 / ref2))


def test_discrete_exact_solution_needs_every_data_term():
    """The exactness above is not automatic: dropping the streamline-diffusion part
    delta (d_t w + d_beta w) of the f functional, or the f functional altogether,
    moves the solution away from u."""
    w = _discrete_exact_workload(1, 1, 4, nstrips=1)
    P = Problem(w)
    b_full = strip.rhs(P, 1, strip.initial_coefficients(P), 1)
    f_part = P.apply(strip.project_in_time(P, w.f, 0.0), P.data_terms())
    Mt = P.Mt
    S = P.spatial_ops()
    plain = [(c * Mt, X, V) for c, X, V in S["M"]]             # (f, w) only
    f_plain = P.apply(strip.project_in_time(P, w.f, 0.0), plain)
    ref = _legendre_slices(P, w.exact, 0.0, w.dt, P.R)
    uref = np.concatenate([np.stack([ref[s][o:o + n] for s in range(P.R)]).ravel()
                           for o, n in zip(np.cumsum([0] + [P.nx(a) * P.nv(b) for a, b in P.upper])[:-1],
                                           [P.nx(a) * P.nv(b) for a, b in P.upper])])
    assert np.linalg.norm(P.apply(uref) - b_full) < 1e-11 * np.linalg.norm(b_full)
    for b_bad in (b_full - f_part + f_plain, b_full - f_part):
        assert np.linalg.norm(P.apply(uref) - b_bad) > 1e-3 * np.linalg.norm(b_full)


@pytest.mark.parametrize("r", [0, 1])
def test_forced_convergence_c1(r):
    """c1 with a reaction sigma = 0.5 and the forcing f = sigma u that keeps
    sin(2 pi (x - v t)) exp(-4 v^2) exact: the error at the final time falls
    with every level (the convergence theorem, thm:convergence: order r + 1/2
    in the SD norm; less in L2 near the time-step floor)."""
    errs = []
    for L in (4, 5, 6):
        w = config_c1()
        w.noise = 0.0
        w.L = L
        w.delta = 0.5 * min(1.0 / 2 ** L, 2.0 / 2 ** L)
        w.r = r
        w.sigma = [(0.5, (), ())]
        ex = w.exact
        w.f = lambda t, X, V, ex=ex: 0.5 * ex(t, X, V)
        P = Problem(w)
        sols, st = strip.march(P, tol=1e-11)
        assert all(s["rel"] <= 1e-11 for s in st)
        T = w.nstrips * w.dt
        exT = strip.interpolate(P, lambda X, V: ex(T, X, V))
        e = strip.trace_right(P, sols[-1], P.R) - exT
        errs.append(np.sqrt(e @ P.apply_mass(e)) / np.sqrt(exT @ P.apply_mass(exT)))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[0] / errs[2] > 3.0, errs
    assert errs[2] < 0.02, errs


# --- Sect. 4.3: the grid-problem preconditioner (mass inverses) ---------------------

from oracle import gridprec  # noqa: E402


def _mass_levels(kind, L):
    w = config_tiny(kind)
    w.L = L
    P = Problem(w)
    return P, [P.factor("x", gridprec.MASS, l, l).toarray() for l in range(w.lmin, L + 1)]


@pytest.mark.parametrize("kind,L", [("d1", 5), ("d1p", 5), ("d2", 3), ("d3", 2)])
def test_jacobi_scaled_mass_spectrum(kind, L):
    """The eigenvalues of D^-1 M of the P1 mass matrix lie in [1/2, 1 + d/2] (the
    Jacobi-scaled element mass matrix (I + 1 1^T)/2 of a d-simplex has exactly these
    two eigenvalues), and the finest level comes close to both ends."""
    P, Ms = _mass_levels(kind, L)
    lo, hi = gridprec.interval(P.w.x.d)
    for M in Ms:
        D = np.diag(M)
        lam = np.linalg.eigvalsh(M / np.sqrt(np.outer(D, D)))
        assert lam.min() >= lo - 1e-12 and lam.max() <= hi + 1e-12, (lam.min(), lam.max())
    assert lam.max() > 0.8 * hi and lam.min() < 0.8


def _cheb_three_term(M, b, k, d):
    """Chebyshev semi-iteration in its three-term form (Varga / Golub-Van Loan):
    x_1 = z_0/theta, x_{j+1} = w_{j+1}(x_j + z_j/theta) + (1 - w_{j+1}) x_{j-1},
    z_j = D^-1 (b - M x_j), w_{j+1} = 2 s T_j(s) / T_{j+1}(s), s = theta/delta."""
    lo, hi = gridprec.interval(d)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    s = theta / delta
    T = [1.0, s]
    for _ in range(k + 1):
        T.append(2 * s * T[-1] - T[-2])
    D = np.diag(M)[:, None]
    xprev = np.zeros_like(b)
    x = b / D / theta
    for j in range(1, k):
        z = (b - M @ x) / D
        w = 2 * s * T[j] / T[j + 1]
        x, xprev = w * (x + z / theta) + (1 - w) * xprev, x
    return x


@pytest.mark.parametrize("kind,L", [("d1", 4), ("d1p", 4), ("d2", 3), ("d3", 2)])
def test_chebyshev_closed_form_equals_the_iteration(kind, L):
    P, Ms = _mass_levels(kind, L)
    d = P.w.x.d
    M = Ms[-1]
    b = np.random.default_rng(4).standard_normal((M.shape[0], 3))
    lo, hi = gridprec.interval(d)
    # one step is the scaled Jacobi step D^-1 b / theta
    C1 = gridprec.chebyshev_inverse(M, 1, d)
    assert np.allclose(C1 @ b, b / np.diag(M)[:, None] / (0.5 * (lo + hi)), rtol=1e-12, atol=0)
    for k in (2, 3, 5, 8):
        ref = _cheb_three_term(M, b, k, d)
        got = gridprec.chebyshev_inverse(M, k, d) @ b
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), k
    # the error falls at least as fast as 1/T_k(theta/delta) and reaches the exact inverse
    xs = np.linalg.solve(M, b)
    Dh = np.sqrt(np.diag(M))[:, None]
    e0 = np.linalg.norm(Dh * xs)
    s = (hi + lo) / (hi - lo)
    for k in (2, 4, 8, 16):
        ek = np.linalg.norm(Dh * (gridprec.chebyshev_inverse(M, k, d) @ b - xs))
        assert ek <= e0 / np.cosh(k * np.arccosh(s)) * (1 + 1e-9), k
    assert np.abs(gridprec.chebyshev_inverse(M, 40, d) @ b - xs).max() <= 1e-12 * np.abs(xs).max()


@pytest.mark.parametrize("kind", ["d1", "d2"])
def test_exact_grid_preconditioner_inverts_its_factors(kind):
    """sweeps = -1: P_l^-1 followed by the forward product (Tt + delta Ct + Gt) (x) M^x (x) M^v
    gives back the input on every grid of both diagonals."""
    w = config_tiny(kind)
    P = Problem(w)
    Tb = gridprec.time_block(P)
    for g in list(P.upper) + list(P.lower):
        U = np.random.default_rng(1).standard_normal((P.R, P.nx(g[0]), P.nv(g[1])))
        Z = gridprec.grid_precond(P, g, U, -1)
        Mx = P.factor("x", gridprec.MASS, g[0], g[0])
        Mv = P.factor("v", gridprec.MASS, g[1], g[1])
        back = np.tensordot(Tb, np.stack([(Mv @ (Mx @ Z[s]).T).T for s in range(P.R)]), axes=(1, 0))
        assert np.abs(back - U).max() <= 1e-11 * np.abs(U).max(), g
    # sweeps = 0 uses the diagonals only: on a grid with more than one node it differs
    g = P.upper[-1]
    U = np.ones((P.R, P.nx(g[0]), P.nv(g[1])))
    assert np.abs(gridprec.grid_precond(P, g, U, 0) - gridprec.grid_precond(P, g, U, -1)).max() > 1e-3


# --- Sect. 4.2: coefficients that depend on time (m-point time quadrature) -------------

@pytest.mark.parametrize("kind", ["d1", "d2"])
def test_time_quadrature_of_constant_fields_is_the_constant_operator(kind):
    """Coefficients that do not change in time: the quadrature form (per-point factors and
    time matrices) equals the closed-form time blocks, for the operator and both data
    functionals (a wrong weight, point or transposed time matrix breaks it)."""
    w = config_tiny(kind)
    P = Problem(w)
    wt = with_time_fields(config_tiny(kind), lambda t, w=w: (dict(w.xfields), dict(w.vfields)))
    Pt = Problem(wt, t0=0.3)
    u = np.random.default_rng(6).standard_normal(P.ndof)
    for a, b in ((P.apply(u), Pt.apply(u)), (P.apply(u, P.data_terms()), Pt.apply(u, Pt.data_terms())),
                 (P.apply(u, P.inflow_data_terms()), Pt.apply(u, Pt.inflow_data_terms()))):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("d,r,L", [(1, 1, 4), (2, 1, 2)])
def test_time_dependent_discrete_exact_solution(d, r, L):
    w = config_timedep_exact(d, r, L)
    u_prev, R_prev = None, 1
    for j in (1, 2):
        P = Problem(w, t0=(j - 1) * w.dt)
        if u_prev is None:
            u_prev = strip.initial_coefficients(P)
        b = strip.rhs(P, j, u_prev, R_prev)
        U, st = fgmres(P.apply, b, CTPreconditioner(P), tol=1e-13, restart=50, maxit=200)
        assert st["rel"] <= 1e-12
        ref = _legendre_slices(P, w.exact, (j - 1) * w.dt, w.dt, P.R)
        blocks = P.split(U)
        err2 = ref2 = 0.0
        for s in range(P.R):
            us = np.concatenate([bb[s].ravel() for bb in blocks])
            e = us - ref[s]
            err2 += abs(e @ P.apply_mass(e))
            ref2 += abs(ref[s] @ P.apply_mass(ref[s]))
        assert np.sqrt(err2 / ref2) < 1e-10, (j, np.sqrt(err2 / ref2))
        u_prev, R_prev = U, P.R
    # frozen at the strip's start instead, the coefficients miss the exact solution
    w2 = config_timedep_exact(d, r, L)
    w2.tfields = None
    xf, vf = w.tfields(w.dt)
    w2.xfields = xf
    P2 = Problem(w2)
    b = strip.rhs(Problem(w, t0=w.dt), 2, u_prev, P2.R)
    assert np.linalg.norm(P2.apply(U) - b) > 1e-4 * np.linalg.norm(b)


def _periodic_x_transport(kind, r):
    """A periodic-x workload whose only coefficients move along x: beta = (v, 0), sigma = 0,
    so every v-factor of A_{l,l} is a (weighted) mass matrix."""
    if kind == "d1":
        w = config_tiny("d1p")
        w.beta = [(1.0, (), ("v0",)), None]
        w.sigma = []
    else:
        w = config_tiny("d2")
        w.x = Domain(2, (0.0, 0.0), (1.0, 1.0), periodic=True)
        w.beta = [(1.0, (), ("v0",)), (1.0, (), ("v1",)), None, None]
        w.sigma = []
    w.r = r
    return w


@pytest.mark.parametrize("kind,r", [("d1", 0), ("d1", 1), ("d2", 1)])
def test_x_transport_operator_is_exact_on_v_constant_functions(kind, r):
    """Lumping a v-mass matrix keeps its action on the constants, so on functions that are
    constant in v the x-transport operator equals the grid problem's A_{l,l} (every term
    of which it keeps when beta has no v-component and sigma = 0); on other functions it
    differs (the lumping is real)."""
    from oracle import gridprec
    w = _periodic_x_transport(kind, r)
    P = Problem(w)
    rng = np.random.default_rng(12)
    for g in list(P.upper) + list(P.lower):
        T = gridprec.transport_operator(P, g)
        A = P.diag_block(g)
        gx = rng.standard_normal((P.R, P.nx(g[0]), 1))
        u = np.broadcast_to(gx, (P.R, P.nx(g[0]), P.nv(g[1]))).ravel()
        assert np.abs(T @ u - A @ u).max() <= 1e-12 * np.abs(A @ u).max(), g
    g = P.upper[0]
    u = rng.standard_normal(P.R * P.nx(g[0]) * P.nv(g[1]))
    T, A = gridprec.transport_operator(P, g), P.diag_block(g)
    assert np.abs(T @ u - A @ u).max() > 1e-6 * np.abs(A @ u).max()


def test_x_transport_operator_acts_on_fourier_modes_by_its_symbol():
    """On a periodic x-lattice the operator maps exp(i theta.x) (x) e_q to
    P(theta, q) exp(i theta.x) (x) e_q with an R x R matrix P(theta, q): a circulant
    block per v-node (checked on every mode of a small grid)."""
    from oracle import gridprec
    w = _periodic_x_transport("d2", 1)
    P = Problem(w)
    g = (2, 0)
    T = gridprec.transport_operator(P, g).toarray()
    n1 = 2 ** g[0]
    nx, nv, R = P.nx(g[0]), P.nv(g[1]), P.R
    X = np.indices((n1, n1)).reshape(2, -1).T
    for m0 in range(n1):
        for m1 in range(n1):
            th = 2 * np.pi * np.array([m0, m1]) / n1
            mode = np.exp(1j * (X @ th))
            for q in range(nv):
                for s in range(R):
                    u = np.zeros((R, nx, nv), complex)
                    u[s, :, q] = mode
                    y = (T @ u.ravel()).reshape(R, nx, nv)
                    assert np.abs(np.delete(y, q, axis=2)).max() < 1e-12
                    coef = y[:, :, q] / mode[None, :]
                    assert np.abs(coef - coef[:, :1]).max() < 1e-12
