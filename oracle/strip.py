"""Right-hand side b_j and strip-by-strip time stepping (eq:weak_form_j).

  b_j(w) = int_{I_j} (f, w + delta (d_t w + d_beta w)) dt
           + int_{I_j} int_{inflow} |beta.n| g w dt          ( = -<g, w>_{Gamma^-} )
           + (U_{j-1}^-, w_{j-1}^+),          U_0^- = u0.

The system of a strip is singular (Sect. 4.2) and solvable only for a
right-hand side that is one linear functional evaluated on the spanning set.
Data enter therefore as sparse-grid functions: f and g are replaced by their
sparse-grid interpolants (nodal values on both diagonals, combined with the
combination formula), projected in time onto P^r by Gauss-Legendre quadrature
with r+2 points; the three functionals are then products of sub-operators of
the Kronecker form with those coefficient vectors.  The jump term uses the
trace U_{j-1}(t_{j-1}^-) = sum_s u_s (Legendre values 1 at the right end) and
w(t_{j-1}^+) = eta_s(-1) = (-1)^s.

Parity: pinned by the tests.  A solution that lies in the discrete space
(affine in x and v, degree <= r in time, r = 0, 1, 2, d = 1 and 2) with its own
f and g as data is reproduced strip after strip to rounding, which fixes every
term of the f functional (including delta (d_t w + d_beta w)), the inflow
functional, the time projection with its (2s+1)/dt factor and the jump term;
the forced c1 problem (reaction plus f = sigma u) converges with the level.
"""
from __future__ import annotations

import numpy as np

from workloads import gauss_legendre_times, random_vector, sample_on_grids

from .ct import CTPreconditioner, combine
from .krylov import fgmres
from .timedg import eta, left_values


def _blocks(P, flat, grids, R):
    out, off = {}, 0
    for (lx, lv) in grids:
        n = P.nx(lx) * P.nv(lv)
        out[(lx, lv)] = flat[off:off + R * n].reshape(R, P.nx(lx), P.nv(lv))
        off += R * n
    return out


def nodal_to_spanning(P, nodal_up, nodal_low, R):
    """Combination of nodal values [R][grid nodes] on both diagonals -> spanning coefficients."""
    up = _blocks(P, nodal_up, P.upper, R)
    low = _blocks(P, nodal_low, P.lower, R)
    return combine(P, up, low)


def _slices_layout(P, per_slice, grids):
    """[R][all nodes of grids] -> [grid][R][nodes] flat."""
    R = len(per_slice)
    out, off = [], 0
    for (lx, lv) in grids:
        n = P.nx(lx) * P.nv(lv)
        out.append(np.stack([s[off:off + n] for s in per_slice]).ravel())
        off += n
    return np.concatenate(out)


def interpolate(P, fn):
    """Sparse-grid interpolant of fn(X, V) as a one-slice spanning vector."""
    w = P.w
    up = sample_on_grids(w, P.upper, fn)
    low = sample_on_grids(w, P.lower, fn)
    return nodal_to_spanning(P, up, low, 1)


def project_in_time(P, fn, t0):
    """Spanning coefficients (R slices) of the P^r(I_j)-projection of the interpolant of fn."""
    w = P.w
    R = P.R
    nq = w.r + 2
    tq, wq = gauss_legendre_times(t0, w.dt, nq)
    xg, _ = np.polynomial.legendre.leggauss(nq)
    vals_up = [sample_on_grids(w, P.upper, fn, t) for t in tq]
    vals_low = [sample_on_grids(w, P.lower, fn, t) for t in tq]
    slices_up, slices_low = [], []
    for s in range(R):
        fac = (2 * s + 1) / w.dt
        e = eta(s, xg)
        slices_up.append(sum(fac * wq[q] * e[q] * vals_up[q] for q in range(nq)))
        slices_low.append(sum(fac * wq[q] * e[q] * vals_low[q] for q in range(nq)))
    return nodal_to_spanning(P, _slices_layout(P, slices_up, P.upper),
                             _slices_layout(P, slices_low, P.lower), R)


def initial_coefficients(P):
    """Spanning coefficients of U_0^- = interpolant of u0 (+ seeded noise if requested)."""
    w = P.w
    u0 = interpolate(P, w.u0) if w.u0 is not None else np.zeros(P.ndof // P.R)
    if w.noise:
        u0 = u0 + w.noise * random_vector(u0.size, w.seed)[0]
    return u0


def trace_right(P, u, R):
    """Coefficients of U(t_j^-) = sum_s u_s eta_s(t_j^-) (all Legendre values are 1)."""
    out, off = [], 0
    for (lx, lv) in P.upper:
        n = P.nx(lx) * P.nv(lv)
        blk = u[off:off + R * n].reshape(R, n)
        out.append(blk.sum(axis=0))
        off += R * n
    return np.concatenate(out)


def jump_rhs(P, u_prev, R_prev):
    m = P.apply_mass(trace_right(P, u_prev, R_prev))
    lv = left_values(P.w.r)
    out, off = [], 0
    for (lx, lvv) in P.upper:
        n = P.nx(lx) * P.nv(lvv)
        out.append(np.outer(lv, m[off:off + n]).ravel())
        off += n
    return np.concatenate(out)


def data_rhs(P, j):
    """Functionals of f and g on strip j (1-based)."""
    w = P.w
    t0 = (j - 1) * w.dt
    b = np.zeros(P.ndof)
    if w.f is not None:
        b += P.apply(project_in_time(P, w.f, t0), P.data_terms())
    if w.g is not None and P.inflow_data_terms():
        b += P.apply(project_in_time(P, w.g, t0), P.inflow_data_terms())
    return b


def rhs(P, j, u_prev, R_prev):
    return jump_rhs(P, u_prev, R_prev) + data_rhs(P, j)


def march(P, nstrips=None, tol=1e-10, restart=50, maxit=400, ct=None, verbose=False):
    """Solve strips 1..nstrips in sequence; returns the list of strip solutions and stats."""
    w = P.w
    nstrips = w.nstrips if nstrips is None else nstrips
    ct = ct or CTPreconditioner(P)
    u_prev, R_prev = initial_coefficients(P), 1
    sols, stats = [], []
    for j in range(1, nstrips + 1):
        b = rhs(P, j, u_prev, R_prev)
        u, st = fgmres(P.apply, b, ct, tol=tol, restart=restart, maxit=maxit)
        if verbose:
            print(f"strip {j}: iters {st['iters']} rel {st['rel']:.2e}")
        sols.append(u)
        stats.append(st)
        u_prev, R_prev = u, P.R
    return sols, stats
