"""O2: the Kronecker-factored space-time operator of one strip (Sect. 4.1-4.2).

A function of P^r(I_j, V_L) is stored by its spanning-set coefficients
(eq:spanningset): one block per upper-diagonal grid l = (lx, lv), each block a
[r+1][n_x][n_v] array (the last index fastest).  The system (eq:Adelta) has
blocks A_{l,l'}; for time-independent coefficients the block formula of
Sect. 4.2 reads

  A_{l,l'} = (Tt + delta Ct + Gt) (x) M + delta Tt (x) T^T + delta Tt^T (x) (T + K)
             + Mt (x) (T + delta C + K + delta K~ - G)

where every spatial matrix is a short sum of Kronecker products of factors on
Omega^(1) and Omega^(2) (separable coefficients, Sect. 4.2).  Reading: the
printed formula carries K~ without delta; expanding (sigma v, delta d_beta w)
from (eq:weak_form_j) gives delta K~, which is used here.

Inflow term: -G = int over the inflow boundary of |beta.n| phi' phi.  On a
face whose normal velocity is s*a(x)*b(v) the weight (beta.n)^- splits exactly
into (s a)^+ b^- + (s a)^- b^+, each factor being the P1 interpolant of the
kinked nodal values on the finest mesh.

Factors on coarse levels come from the finest one (Sect. 4.2):
  X_{l,l'} = E_{L,l}^T X_{L,L} E_{L,l'}.
The blockwise product [A u]_l = sum_l' A_{l,l'} u_l' applies each Kronecker
term in the order prescribed at the end of Sect. 4.2 (v-factor first when
lx' + lv <= lx + lv', x-factor first otherwise).

Parity: pinned against O1 (brute.py) on small grids, plus kernel vectors,
constant consistency and positive semi-definiteness (tests).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from workloads import grid_levels, lattice_coords, nodal_fields

from .fe import assemble, weight_nodal
from .mesh import Lattice, embedding_chain
from .timedg import time_matrices, time_quadrature

W1 = (1.0, (), None)


def _fkey(kind, weight=W1, a=None, b=None, face=None, trans=False):
    return (kind, weight, a, b, face, trans)


def _T(key):
    k = list(key); k[5] = not k[5]
    return tuple(k)


def _cat(w1, w2):
    return (w1[0] * w2[0], tuple(w1[1]) + tuple(w2[1]), None)


class Problem:
    """One strip's discrete operator for a workload (FP64, scipy.sparse)."""

    def __init__(self, w, t0=0.0):
        self.w = w
        self.d = w.d
        self.R = w.r + 1
        self.t0 = t0
        self.fx, self.fv = nodal_fields(w)
        self.upper, self.lower = grid_levels(w)
        self._E = {}
        self._fine = {}
        self._fac = {}
        self.Mt, self.Tt, self.Ct, self.Gt = time_matrices(w.r, w.dt)
        self.tq = None
        if w.tfields is not None:
            # coefficients that depend on time: the fields at the quadrature points of
            # the strip [t0, t0 + dt], registered as "name@mu"
            m = w.tquad if w.tquad else w.r + 2
            self.tq = time_quadrature(w.r, w.dt, m)
            X = lattice_coords(w.x, w.L)
            V = lattice_coords(w.v, w.L)
            for mu, tau in enumerate(self.tq["tau"]):
                xf, vf = w.tfields(t0 + 0.5 * w.dt * (tau + 1.0))
                for k, fn in xf.items():
                    self.fx[f"{k}@{mu}"] = np.ascontiguousarray(fn(X), dtype=np.float64)
                for k, fn in vf.items():
                    self.fv[f"{k}@{mu}"] = np.ascontiguousarray(fn(V), dtype=np.float64)
        self.terms = self.build_terms()
        self.sizes = [self.nx(lx) * self.nv(lv) for lx, lv in self.upper]
        self.offsets = np.concatenate([[0], np.cumsum([self.R * s for s in self.sizes])])
        self.ndof = int(self.offsets[-1])

    # -- domains -------------------------------------------------------------
    def dom(self, which):
        return self.w.x if which == "x" else self.w.v

    def lat(self, which, level):
        D = self.dom(which)
        return Lattice(D.d, D.lo, D.hi, level, D.periodic)

    def nx(self, l):
        return self.lat("x", l).n

    def nv(self, l):
        return self.lat("v", l).n

    def E(self, which, lf, lc):
        key = (which, lf, lc)
        if key not in self._E:
            D = self.dom(which)
            self._E[key] = embedding_chain(D.d, D.lo, D.hi, D.periodic, lf, lc)
        return self._E[key]

    # -- factors ---------------------------------------------------------------
    def fine_factor(self, which, key):
        base = tuple(key[:5]) + (False,)
        ck = (which, base)
        if ck not in self._fine:
            kind, weight, a, b, face, _ = base
            lat = self.lat(which, self.w.L)
            fields = self.fx if which == "x" else self.fv
            scale, wf = weight_nodal(fields, weight, lat.n)
            self._fine[ck] = assemble(lat, kind, wf, scale=scale, a=a, b=b, face=face).tocsr()
        X = self._fine[ck]
        return X.T.tocsr() if key[5] else X

    def factor(self, which, key, lrow, lcol):
        """X_{lrow,lcol} = E_{L,lrow}^T X_{L,L} E_{L,lcol} (Sect. 4.2)."""
        ck = (which, key, lrow, lcol)
        if ck not in self._fac:
            L = self.w.L
            X = self.fine_factor(which, key)
            self._fac[ck] = (self.E(which, L, lrow).T @ X @ self.E(which, L, lcol)).tocsr()
        return self._fac[ck]

    # -- the operator as a list of Kronecker terms -----------------------------
    def specs_at(self, mu):
        """beta and sigma of the workload with every field name taken at quadrature point mu."""
        def ren(names):
            return tuple(f"{k}@{mu}" for k in names)
        beta = [None if b is None else (b[0], ren(b[1]), ren(b[2])) for b in self.w.beta]
        sigma = [(c, ren(P), ren(Q)) for c, P, Q in self.w.sigma]
        return beta, sigma

    def spatial_ops(self, beta=None, sigma=None):
        d = self.d
        w = self.w
        beta = w.beta if beta is None else beta
        sigma = w.sigma if sigma is None else sigma
        M = [(1.0, _fkey("mass"), _fkey("mass"))]
        T, C, K, Kt, Gm = [], [], [], [], []
        for c in range(2 * d):
            if beta[c] is None:
                continue
            s, A, B = beta[c]
            if c < d:
                T.append((s, _fkey("deriv", (1.0, A, None), a=c), _fkey("mass", (1.0, B, None))))
            else:
                T.append((s, _fkey("mass", (1.0, A, None)), _fkey("deriv", (1.0, B, None), a=c - d)))
        # C_{k,k'} = (beta.grad phi_k', beta.grad phi_k) = sum_{c,c2} beta_c beta_c2 (d_c phi', d_c2 phi)
        for c in range(2 * d):
            for c2 in range(2 * d):
                if beta[c] is None or beta[c2] is None:
                    continue
                s1, A1, B1 = beta[c]
                s2, A2, B2 = beta[c2]
                wa = (1.0, tuple(A1) + tuple(A2), None)
                wb = (1.0, tuple(B1) + tuple(B2), None)
                if c < d and c2 < d:
                    X, V = _fkey("stiff", wa, a=c, b=c2), _fkey("mass", wb)
                elif c < d <= c2:
                    X, V = _fkey("deriv", wa, a=c), _T(_fkey("deriv", wb, a=c2 - d))
                elif c2 < d <= c:
                    X, V = _T(_fkey("deriv", wa, a=c2)), _fkey("deriv", wb, a=c - d)
                else:
                    X, V = _fkey("mass", wa), _fkey("stiff", wb, a=c - d, b=c2 - d)
                C.append((s1 * s2, X, V))
        for (sc, P, Q) in sigma:
            K.append((sc, _fkey("mass", (1.0, P, None)), _fkey("mass", (1.0, Q, None))))
            # K~_{k,k'} = (sigma phi_k', beta.grad phi_k)
            for c in range(2 * d):
                if beta[c] is None:
                    continue
                s, A, B = beta[c]
                wa = (1.0, tuple(P) + tuple(A), None)
                wb = (1.0, tuple(Q) + tuple(B), None)
                if c < d:
                    Kt.append((sc * s, _T(_fkey("deriv", wa, a=c)), _fkey("mass", wb)))
                else:
                    Kt.append((sc * s, _fkey("mass", wa), _T(_fkey("deriv", wb, a=c - d))))
        # -G: inflow faces of the product domain
        for axis in range(d):
            for which in ("x", "v"):
                D = self.dom(which)
                if D.periodic:
                    continue
                c = axis if which == "x" else d + axis
                if beta[c] is None:
                    continue
                s, A, B = beta[c]
                for side in (0, 1):
                    sgn = -1.0 if side == 0 else 1.0
                    for ka, kb in (("pos", "neg"), ("neg", "pos")):
                        wa = (sgn * s, tuple(A), ka)
                        wb = (1.0, tuple(B), kb)
                        if which == "x":
                            X = _fkey("face", wa, face=(axis, side))
                            V = _fkey("mass", wb)
                        else:
                            X = _fkey("mass", wa)
                            V = _fkey("face", wb, face=(axis, side))
                        Gm.append((1.0, X, V))
        return dict(M=M, T=T, C=C, K=K, Kt=Kt, Gm=Gm)

    def build_terms(self):
        """Kronecker terms (time matrix (R,R), x-factor key, v-factor key) of A."""
        w = self.w
        dl = w.delta

        def tr(ops):
            return [(c, _T(X), _T(V)) for c, X, V in ops]

        if self.tq is not None:
            # Sect. 4.2, block formula with an m-point time quadrature: per point mu the
            # spatial factors of the coefficients at tau_mu and the time matrices
            # w_mu eta_s'(tau_mu) eta_s(tau_mu) (and derivatives); G^t once
            groups = [(self.Gt, self.spatial_ops()["M"])]
            for mu in range(len(self.tq["tau"])):
                S = self.spatial_ops(*self.specs_at(mu))
                Mm, Tm, Cm = self.tq["M"][mu], self.tq["T"][mu], self.tq["C"][mu]
                groups += [
                    (Tm + dl * Cm, S["M"]),
                    (dl * Tm, tr(S["T"])),
                    (dl * Tm.T, S["T"] + S["K"]),
                    (Mm, S["T"] + [(dl * c, X, V) for c, X, V in S["C"]] + S["K"]
                     + [(dl * c, X, V) for c, X, V in S["Kt"]] + S["Gm"]),
                ]
            return self._collect(groups)
        S = self.spatial_ops()
        groups = [
            (self.Tt + dl * self.Ct + self.Gt, S["M"]),
            (dl * self.Tt, tr(S["T"])),
            (dl * self.Tt.T, S["T"] + S["K"]),
            (self.Mt, S["T"] + [(dl * c, X, V) for c, X, V in S["C"]] + S["K"]
             + [(dl * c, X, V) for c, X, V in S["Kt"]] + S["Gm"]),
        ]
        return self._collect(groups)

    @staticmethod
    def _collect(groups):
        terms = []
        for Tm, ops in groups:
            if not np.any(Tm):
                continue
            for c, X, V in ops:
                terms.append((c * Tm, X, V))
        return terms

    def mass_terms(self):
        """The cross-grid L2 inner product (phi', phi) of the spanning set, one time slice."""
        return [(np.ones((1, 1)), _fkey("mass"), _fkey("mass"))]

    def data_terms(self):
        """b_f(w) = int (f, w + delta (d_t w + d_beta w)) for f in P^r(I_j, V_L)."""
        dl = self.w.delta
        if self.tq is not None:
            S0 = self.spatial_ops()
            groups = [(self.Mt + dl * self.Tt.T, S0["M"])]
            for mu in range(len(self.tq["tau"])):
                S = self.spatial_ops(*self.specs_at(mu))
                groups.append((dl * self.tq["M"][mu], [(c, _T(X), _T(V)) for c, X, V in S["T"]]))
            return self._collect(groups)
        S = self.spatial_ops()
        ops = [(self.Mt + dl * self.Tt.T, S["M"])] + [(dl * self.Mt, [(c, _T(X), _T(V)) for c, X, V in S["T"]])]
        out = []
        for Tm, lst in ops:
            if not np.any(Tm):
                continue
            for c, X, V in lst:
                out.append((c * Tm, X, V))
        return out

    def inflow_data_terms(self):
        """b_g(w) = int over the inflow boundary of |beta.n| g w, for g in P^r(I_j, V_L)."""
        if self.tq is not None:
            groups = [(self.tq["M"][mu], self.spatial_ops(*self.specs_at(mu))["Gm"])
                      for mu in range(len(self.tq["tau"]))]
            return self._collect(groups)
        S = self.spatial_ops()
        return [(c * self.Mt, X, V) for c, X, V in S["Gm"]]

    # -- application ---------------------------------------------------------------
    def block_apply(self, terms, lrow, lcol, ucol, R_in=None):
        """sum_terms (Tm (x) X_{lx,lx'} (x) V_{lv,lv'}) u_{l'} in the paper's factor order."""
        (lx, lv), (lx2, lv2) = lrow, lcol
        nxr, nvr, nxc, nvc = self.nx(lx), self.nv(lv), self.nx(lx2), self.nv(lv2)
        Rin = ucol.shape[0]
        Rout = terms[0][0].shape[0]
        y = np.zeros((Rout, nxr, nvr))
        for Tm, X, V in terms:
            Xm = self.factor("x", X, lx, lx2)
            Vm = self.factor("v", V, lv, lv2)
            Z = np.empty((Rin, nxr, nvr))
            for s in range(Rin):
                U = ucol[s]
                if lx2 + lv <= lx + lv2:           # v-factor first
                    Z[s] = Xm @ (Vm @ U.T).T
                else:                              # x-factor first
                    Z[s] = (Vm @ (Xm @ U).T).T
            y += np.tensordot(Tm, Z, axes=(1, 0))
        return y

    def split(self, u, R=None):
        R = self.R if R is None else R
        out = []
        off = 0
        for (lx, lv) in self.upper:
            n = self.nx(lx) * self.nv(lv)
            out.append(u[off:off + R * n].reshape(R, self.nx(lx), self.nv(lv)))
            off += R * n
        return out

    def apply(self, u, terms=None, R_in=None):
        """[A u]_l = sum_{l'} A_{l,l'} u_{l'} (Sect. 4.2), blockwise."""
        terms = self.terms if terms is None else terms
        Rin = terms[0][0].shape[1]
        Rout = terms[0][0].shape[0]
        blocks = self.split(np.asarray(u, float), Rin)
        out = []
        for l in self.upper:
            y = np.zeros((Rout, self.nx(l[0]), self.nv(l[1])))
            for l2, ub in zip(self.upper, blocks):
                y += self.block_apply(terms, l, l2, ub)
            out.append(y.ravel())
        return np.concatenate(out)

    def apply_mass(self, u1):
        """Cross-grid mass product for a one-slice vector."""
        return self.apply(u1, self.mass_terms())

    # -- assembled matrices (small problems) ------------------------------------------
    def assembled_block(self, terms, lrow, lcol):
        (lx, lv), (lx2, lv2) = lrow, lcol
        out = None
        for Tm, X, V in terms:
            blk = sp.kron(sp.csr_matrix(Tm), sp.kron(self.factor("x", X, lx, lx2),
                                                      self.factor("v", V, lv, lv2)))
            out = blk if out is None else out + blk
        return out.tocsr()

    def assembled(self, terms=None):
        terms = self.terms if terms is None else terms
        rows = [[self.assembled_block(terms, l, l2) for l2 in self.upper] for l in self.upper]
        return sp.bmat(rows).tocsr()

    def diag_block(self, grid):
        """A_{l,l} for any component grid l (upper or lower diagonal)."""
        return self.assembled_block(self.terms, grid, grid)
