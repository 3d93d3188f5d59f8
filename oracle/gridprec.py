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

The x-transport preconditioner at the end (periodic x) is an extension: the
x-advection and x-streamline-diffusion part of A_{l,l} with the v-mass
matrices lumped, block-circulant in x for every v-node.

Parity: pinned by the tests -- the spectrum of D^-1 M lies in the interval
for d = 1, 2, 3 (periodic or not); the closed form equals a textbook
three-term Chebyshev iteration run step by step; one step is D^-1 b / theta;
many steps reach the exact inverse; the exact form inverts the forward
product of the three factors; the transport operator acts on every Fourier mode
of a periodic x-lattice (times a v-node indicator) by its stencil symbol.
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


# --- x-transport preconditioner for periodic x (an extension beyond Sect. 4.3) ------------

def transport_operator(P, grid):
    """The part of A_{l,l} that transports along x, with the v-mass matrices lumped:

        P_l = (Tt + d Ct + Gt) (x) M (x) L0 + d Tt (x) sum_i D_i^T (x) L_i
              + d Tt^T (x) sum_i D_i (x) L_i + Mt (x) (sum_i D_i (x) L_i + d sum_ij S_ij (x) L_ij),

    d the streamline-diffusion parameter, D_i and S_ij the x-derivative and x-stiffness
    factors of level lx, L0 = diag(M^v 1), L_i = diag(M^v[b_i] 1) and L_ij = diag(M^v[b_i b_j] 1)
    the lumped v-masses (row sums) weighted with the v-fields b_i of beta's x-components
    beta_i = s_i b_i(v) (which must not depend on x).  The v-transport, reaction and
    inflow terms of A_{l,l} are left out.  On a periodic x-lattice every v-node's block
    is a circulant matrix in x.  Returns the sparse matrix on the grid's [R][n_x][n_v] layout."""
    import scipy.sparse as sp
    lx, lv = grid
    w = P.w
    dl = w.delta
    d = P.d
    Mx = P.factor("x", MASS, lx, lx)
    mv = lambda names: P.factor("v", _fkey("mass", (1.0, tuple(names), None)), lv, lv) @ np.ones(P.nv(lv))
    xc = []
    for c in range(d):
        b = w.beta[c]
        if b is None:
            continue
        s, A, Bn = b
        assert len(A) == 0, "the x-components of beta must not depend on x"
        xc.append((c, s, tuple(Bn)))
    L0 = sp.diags(mv(()))
    T = None
    for c, s, Bn in xc:
        Dc = P.factor("x", _fkey("deriv", (1.0, (), None), a=c), lx, lx)
        t = s * sp.kron(Dc, sp.diags(mv(Bn)))
        T = t if T is None else T + t
    Cm = None
    for c, s, Bn in xc:
        for c2, s2, Bn2 in xc:
            S = P.factor("x", _fkey("stiff", (1.0, (), None), a=c, b=c2), lx, lx)
            t = s * s2 * sp.kron(S, sp.diags(mv(Bn + Bn2)))
            Cm = t if Cm is None else Cm + t
    R = P.R
    Tt, Ct, Gt, Mt = P.Tt, P.Ct, P.Gt, P.Mt
    out = sp.kron(sp.csr_matrix(Tt + dl * Ct + Gt), sp.kron(Mx, L0))
    if T is not None:
        out = out + sp.kron(sp.csr_matrix(dl * Tt), T.T) + sp.kron(sp.csr_matrix(dl * Tt.T), T)
        out = out + sp.kron(sp.csr_matrix(Mt), T + (dl * Cm if Cm is not None else 0 * T))
    return out.tocsr()


def transport_precond(P, grid, U):
    """P_l^-1 U by a direct sparse solve (the plain definition); U of shape (R, n_x, n_v)."""
    import scipy.sparse.linalg as spla
    A = transport_operator(P, grid)
    return spla.spsolve(A.tocsc(), U.ravel()).reshape(U.shape)


def transport_precond_all(P, vec):
    out, off = [], 0
    for g in list(P.upper) + list(P.lower):
        n = P.R * P.nx(g[0]) * P.nv(g[1])
        out.append(transport_precond(P, g, vec[off:off + n].reshape(P.R, P.nx(g[0]), P.nv(g[1]))).ravel())
        off += n
    return np.concatenate(out)
