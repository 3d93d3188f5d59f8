"""The combination-technique preconditioner: the body of Algorithm 1 (Sect. 4.3).

Given a residual r in spanning coefficients (upper grids, |l|_1 = L + lmin),
    1. solve A_{l,l} dU_l = r_l on every upper grid,
    2. for every lower grid (lx, lv) (|l|_1 = L + lmin - 1) restrict the residual
       of the upper grid (lx+1, lv) in x: r_l = (Id (x) E^(1)_{lx+1,lx}^T (x) Id) r,
       and solve A_{l,l} dU_l = r_l,
    3. combine on the upper grids: dU_l - (Id (x) E^(1)_{lx,lx-1} (x) Id) dU_{(lx-1,lv)}
       for lx > lmin, dU_l for lx = lmin.
The paper solves the grid problems (eq:Adeltall) by preconditioned GMRES; here
they are solved directly (sparse LU of the assembled A_{l,l}), i.e. exactly, so
this is the preconditioner that any inner solve converges to.

The same combination step turns nodal interpolants on the two diagonals into
the spanning coefficients of the sparse-grid interpolant (the combination
technique is exact for interpolation, Sect. 4.3).

Parity: pinned by the tests (one-grid sparse grid gives A^{-1}; linearity;
P_CT(A u) = u for u in V_lmin (x) V_lmin, the space every component grid
contains, because each grid problem is A restricted to its component space;
reproduction of the sparse-grid interpolant).  For general residuals the
preconditioner has no closed form beyond these steps.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


class CTPreconditioner:
    def __init__(self, P, inner="direct"):
        self.P = P
        self.inner = inner
        self._lu = {}

    def solve_grid(self, grid, rhs):
        if grid not in self._lu:
            self._lu[grid] = spla.splu(self.P.diag_block(grid).tocsc())
        return self._lu[grid].solve(rhs)

    def restrict_x(self, grid_fine, arr):
        """(Id (x) E^T (x) Id) from x-level lx+1 to lx; arr has shape (R, nx_fine, nv)."""
        lx, lv = grid_fine
        E = self.P.E("x", lx, lx - 1)
        return np.stack([E.T @ a for a in arr])

    def prolong_x(self, grid_coarse, arr):
        lx, lv = grid_coarse
        E = self.P.E("x", lx + 1, lx)
        return np.stack([E @ a for a in arr])

    def __call__(self, r):
        P = self.P
        R = P.R
        rb = dict(zip(P.upper, P.split(np.asarray(r, float))))
        du_up = {}
        for g in P.upper:
            du_up[g] = self.solve_grid(g, rb[g].ravel()).reshape(rb[g].shape)
        du_low = {}
        for (lx, lv) in P.lower:
            rl = self.restrict_x((lx + 1, lv), rb[(lx + 1, lv)])
            du_low[(lx, lv)] = self.solve_grid((lx, lv), rl.ravel()).reshape(rl.shape)
        return combine(P, du_up, du_low)


def combine(P, up, low):
    """Spanning coefficients of sum_upper f_l - sum_lower f_l (the combination formula)."""
    out = []
    for (lx, lv) in P.upper:
        z = up[(lx, lv)].copy()
        if lx > P.w.lmin:
            E = P.E("x", lx, lx - 1)
            z -= np.stack([E @ a for a in low[(lx - 1, lv)]])
        out.append(z.ravel())
    return np.concatenate(out)
