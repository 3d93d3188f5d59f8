"""The grid-problem preconditioner of Sect. 4.3 (test infrastructure, CPU, FP64).

Every grid problem A_{l,l} dU_l = r_l (eq:Adeltall) is solved by GMRES,
preconditioned with the inverse of the dominant part of A_{l,l}:

    P_l = (Tt + delta Ct + Gt) (x) M^x_{lx} (x) M^v_{lv},

the time block of the mass term times the two spatial mass matrices (the
term of (eq:Adelta) that carries no factor dt).  The three factors act on
different axes, so P_l^-1 is the product of the three inverses.

The mass inverses come in three forms, selected by `sweeps`:
  * sweeps = -1: the exact inverse (a dense solve here);
  * sweeps =  0: the diagonal of the mass matrix instead of the matrix;
  * sweeps =  k: k steps of Chebyshev acceleration of the Jacobi splitting
    D = diag(M), started from zero, for the spectrum interval [1/2, 1 + d/2]
    of D^-1 M (d the dimension of the domain).

The k-step Chebyshev iterate has a closed form (the defining property of the
method, e.g. Saad, Iterative Methods for Sparse Linear Systems, Sect. 12.3):
its error is e_k = q_k(D^-1 M) e_0 with the scaled Chebyshev polynomial
q_k(lam) = T_k((theta - lam)/delta) / T_k(theta/delta), theta and delta the
centre and half-width of the interval.  From x_0 = 0 (e_0 = M^-1 b) that is

    x_k = D^-1/2 Q diag((1 - q_k(lam_i)) / lam_i) Q^T D^-1/2 b,

with C = D^-1/2 M D^-1/2 = Q diag(lam) Q^T.  This module evaluates it that
way, by a dense eigendecomposition; it is meant for small levels.

Parity: pinned by the tests -- the spectrum of D^-1 M lies in the interval
for d = 1, 2, 3 (periodic or not); the closed form equals a textbook
three-term Chebyshev iteration run step by step; one step is D^-1 b / theta;
many steps reach the exact inverse; the exact form inverts the forward
product of the three factors.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as npcheb

from .operator import _fkey

MASS = _fkey("mass")


def interval(d):
    """Spectrum bounds of D^-1 M for the P1 mass matrix on d-simplices."""
    return 0.5, 1.0 + 0.5 * d


def chebyshev_inverse(M, k, d):
    """Dense matrix of the k-step Chebyshev-Jacobi approximation of M^-1 (closed form)."""
    M = np.asarray(M, float)
    D = np.diag(M).copy()
    s = 1.0 / np.sqrt(D)
    C = s[:, None] * M * s[None, :]
    lam, Q = np.linalg.eigh(0.5 * (C + C.T))
    lo, hi = interval(d)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    Tk = npcheb.Chebyshev.basis(k)
    q = Tk((theta - lam) / delta) / Tk(theta / delta)
    g = (1.0 - q) / lam
    return s[:, None] * (Q * g[None, :]) @ Q.T * s[None, :]


def mass_inverse(M, sweeps, d):
    M = np.asarray(M, float)
    if sweeps < 0:
        return np.linalg.inv(M)
    if sweeps == 0:
        return np.diag(1.0 / np.diag(M))
    return chebyshev_inverse(M, sweeps, d)


def time_block(P):
    return P.Tt + P.w.delta * P.Ct + P.Gt


def grid_precond(P, grid, U, sweeps):
    """P_l^-1 U for one component grid l = (lx, lv); U has shape (R, n_x, n_v)."""
    lx, lv = grid
    Mx = P.factor("x", MASS, lx, lx).toarray()
    Mv = P.factor("v", MASS, lv, lv).toarray()
    Cx = mass_inverse(Mx, sweeps, P.w.x.d)
    Cv = mass_inverse(Mv, sweeps, P.w.v.d)
    Z = np.stack([Cx @ U[s] @ Cv.T for s in range(U.shape[0])])
    return np.tensordot(np.linalg.inv(time_block(P)), Z, axes=(1, 0))


def grid_precond_all(P, vec, sweeps):
    """P_l^-1 on the grid-problem layout: every upper grid, then every lower grid,
    each an [R][n_x][n_v] block."""
    out, off = [], 0
    for g in list(P.upper) + list(P.lower):
        n = P.R * P.nx(g[0]) * P.nv(g[1])
        U = vec[off:off + n].reshape(P.R, P.nx(g[0]), P.nv(g[1]))
        out.append(grid_precond(P, g, U, sweeps).ravel())
        off += n
    return np.concatenate(out)
