"""O1: brute-force assembly of the strip matrix A^(delta) of (eq:Adelta).

Every entry is the bilinear form a_j^(delta) of (eq:weak_form_j) evaluated on two
spanning functions eta_s'(t) phi_{l'x,k'x}(x) phi_{l'v,k'v}(v) (trial) and
eta_s(t) phi_{lx,kx}(x) phi_{lv,kv}(v) (test):

  a_j(v, w) = int_{I_j} (d_t v + beta.grad v + sigma v, w + delta (d_t w + beta.grad w))
              + int_{I_j} int_{inflow} |beta.n| v w  +  (v(t_{j-1}), w(t_{j-1})).

The integrals are computed by quadrature on the finest product mesh (every
coarse hat function is linear on each finest simplex) with the basis functions
and the coefficients evaluated pointwise; beta and sigma are the P1 interpolants
of the given nodal fields, and the inflow weight max(-beta.n, 0) is evaluated
pointwise.  No Kronecker factorisation, factor matrix or embedding matrix is
used, which makes this tier an independent check of O2.

Parity: this is a definition (the weak form itself); only sizes that fit a
dense matrix are supported.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from workloads import grid_levels, nodal_fields

from .mesh import Lattice
from .quad import simplex_rule
from .timedg import deta, eta


def _lat(dom, level):
    return Lattice(dom.d, dom.lo, dom.hi, level, dom.periodic)


def _field_at(dom, L, nodal, pts):
    vals, _ = _lat(dom, L).eval(pts)
    return vals @ nodal


def _factor_values(dom, L, fields, names, pts, scale=1.0):
    out = np.full(pts.shape[0], float(scale))
    for k in names:
        out = out * _field_at(dom, L, fields[k], pts)
    return out


def _domain_rule(dom, L, n):
    idx, xyz = _lat(dom, L).simplices()
    return simplex_rule(xyz, n)


def _face_rule(dom, L, axis, side, n):
    fidx, fxyz = _lat(dom, L).boundary_facets(axis, side)
    return simplex_rule(fxyz, n)


class Brute:
    def __init__(self, w, nq_x=None, nq_v=None):
        self.w = w
        self.d = w.d
        self.R = w.r + 1
        self.fx, self.fv = nodal_fields(w)
        self.upper, _ = grid_levels(w)
        self.nq_x = nq_x or 4
        self.nq_v = nq_v or 4

    def _basis(self, dom, level, pts):
        return _lat(dom, level).eval(pts)

    def _beta_parts(self, px, pv):
        """beta_c at product points as (x-part, v-part) vectors."""
        w = self.w
        parts = []
        for c in range(2 * self.d):
            if w.beta[c] is None:
                parts.append(None)
                continue
            s, A, B = w.beta[c]
            parts.append((_factor_values(w.x, w.L, self.fx, A, px, s),
                          _factor_values(w.v, w.L, self.fv, B, pv)))
        return parts

    def _sigma(self, px, pv):
        w = self.w
        out = np.zeros((px.shape[0], pv.shape[0]))
        for sc, P, Q in w.sigma:
            out += np.outer(_factor_values(w.x, w.L, self.fx, P, px, sc),
                            _factor_values(w.v, w.L, self.fv, Q, pv))
        return out.ravel()

    def _grid_mats(self, px, pv):
        """Per upper grid: B (values), BG (beta.grad) at the product points."""
        w = self.w
        bp = self._beta_parts(px, pv)
        out = []
        for lx, lv in self.upper:
            Bx, Gx = self._basis(w.x, lx, px)
            Bv, Gv = self._basis(w.v, lv, pv)
            B = sp.kron(Bx, Bv, format="csr")
            BG = None
            for c in range(2 * self.d):
                if bp[c] is None:
                    continue
                ax, bv = bp[c]
                if c < self.d:
                    term = sp.kron(sp.diags(ax) @ Gx[c], sp.diags(bv) @ Bv, format="csr")
                else:
                    term = sp.kron(sp.diags(ax) @ Bx, sp.diags(bv) @ Gv[c - self.d], format="csr")
                BG = term if BG is None else BG + term
            if BG is None:
                BG = sp.csr_matrix(B.shape)
            out.append((B, BG))
        return out

    def matrix(self):
        """Dense A^(delta) for one strip (upper grids, layout [grid][s][kx][kv])."""
        w = self.w
        R, dl, dt = self.R, w.delta, w.dt
        px_all, wx_all = _domain_rule(w.x, w.L, self.nq_x)
        pv, wv = _domain_rule(w.v, w.L, self.nq_v)
        tq, tw = np.polynomial.legendre.leggauss(w.r + 2)
        ntot = sum(R * _lat(w.x, lx).n * _lat(w.v, lv).n for lx, lv in self.upper)
        A = np.zeros((ntot, ntot))
        chunk = max(1, 200000 // max(1, pv.shape[0]))
        for c0 in range(0, px_all.shape[0], chunk):
            px, wx = px_all[c0:c0 + chunk], wx_all[c0:c0 + chunk]
            mats = self._grid_mats(px, pv)
            sig = self._sigma(px, pv)
            wq = np.outer(wx, wv).ravel()
            for tau, wt in zip(tq, tw):
                wt = wt * dt / 2
                LV, LW = [], []
                for B, BG in mats:
                    SB = sp.diags(sig) @ B
                    for s in range(R):
                        e, de = eta(s, tau), deta(s, tau, dt)
                        LV.append(de * B + e * (BG + SB))
                        LW.append((e + dl * de) * B + dl * e * BG)
                LV = sp.hstack(LV, format="csr")
                LW = sp.hstack(LW, format="csr")
                A += wt * (LW.T @ sp.diags(wq) @ LV).toarray()
            # jump term (v(t_{j-1}^+), w(t_{j-1}^+))
            J = []
            for B, BG in mats:
                for s in range(R):
                    J.append(eta(s, -1.0) * B)
            J = sp.hstack(J, format="csr")
            A += (J.T @ sp.diags(wq) @ J).toarray()
        A += self._inflow(tq, tw)
        return A

    def _inflow(self, tq, tw):
        w = self.w
        R, dt = self.R, w.dt
        ntot = sum(R * _lat(w.x, lx).n * _lat(w.v, lv).n for lx, lv in self.upper)
        A = np.zeros((ntot, ntot))
        for which in ("x", "v"):
            dom = w.x if which == "x" else w.v
            if dom.periodic:
                continue
            for axis in range(self.d):
                c = axis if which == "x" else self.d + axis
                if w.beta[c] is None:
                    continue
                for side in (0, 1):
                    sgn = -1.0 if side == 0 else 1.0
                    if which == "x":
                        px, wx = _face_rule(w.x, w.L, axis, side, self.nq_x)
                        pv, wv = _domain_rule(w.v, w.L, self.nq_v)
                    else:
                        px, wx = _domain_rule(w.x, w.L, self.nq_x)
                        pv, wv = _face_rule(w.v, w.L, axis, side, self.nq_v)
                    bp = self._beta_parts(px, pv)
                    ax, bv = bp[c]
                    bn = sgn * np.outer(ax, bv).ravel()
                    wt_in = np.maximum(-bn, 0.0) * np.outer(wx, wv).ravel()
                    mats = self._grid_mats(px, pv)
                    for tau, wt in zip(tq, tw):
                        wt = wt * dt / 2
                        Bl = []
                        for B, _ in mats:
                            for s in range(R):
                                Bl.append(eta(s, tau) * B)
                        Bl = sp.hstack(Bl, format="csr")
                        A += wt * (Bl.T @ sp.diags(wt_in) @ Bl).toarray()
        return A
