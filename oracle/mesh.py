"""Nested uniform simplicial meshes of a box and their P1 spaces (Sect. 2).

The paper builds nested spaces V_1 ⊂ V_2 ⊂ ... by uniform refinement with
dim V_l ~ 2**(d l).  Here level l of a box has 2**l cells per axis, each cell
split into the d! Kuhn simplices along its main diagonal (the simplex of a
point is fixed by the descending order of its local coordinates).  Halving the
cell size keeps every fine simplex inside one coarse simplex, so the P1 spaces
are nested.  The embedding matrix E_{l+1,l} is obtained here by *evaluating*
the level-l hat functions at the level-(l+1) nodes.

Parity: pinned by the tests (E*1 = 1, partition of unity, Kuhn simplices tile
the box, nodal interpolation reproduces linear functions).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp


class Lattice:
    """One level of a box domain: nodes, Kuhn simplices, P1 evaluation."""

    def __init__(self, d, lo, hi, level, periodic=False):
        self.d = int(d)
        self.lo = np.asarray(lo, float)
        self.hi = np.asarray(hi, float)
        self.level = int(level)
        self.periodic = bool(periodic)
        self.ncell = 2 ** self.level
        self.h = (self.hi - self.lo) / self.ncell
        self.m = self.ncell if self.periodic else self.ncell + 1
        self.shape = (self.m,) * self.d
        self.n = self.m ** self.d

    # -- node numbering ------------------------------------------------------
    def index(self, multi):
        """Linear index of integer multi-indices (..., d); wraps periodic axes."""
        multi = np.asarray(multi)
        if self.periodic:
            multi = np.mod(multi, self.ncell)
        idx = np.zeros(multi.shape[:-1], dtype=np.int64)
        for a in range(self.d):
            idx = idx * self.m + multi[..., a]
        return idx

    def node_multi(self):
        return np.indices(self.shape).reshape(self.d, -1).T

    def node_coords(self):
        return self.lo + self.node_multi() * self.h

    # -- simplices -----------------------------------------------------------
    def simplices(self):
        """Kuhn simplices: (nsimp, d+1) node indices and (nsimp, d+1, d) coordinates."""
        cells = np.indices((self.ncell,) * self.d).reshape(self.d, -1).T
        out_idx, out_xyz = [], []
        for perm in itertools.permutations(range(self.d)):
            verts = [cells.copy()]
            for a in perm:
                nxt = verts[-1].copy()
                nxt[:, a] += 1
                verts.append(nxt)
            V = np.stack(verts, axis=1)                 # (ncells, d+1, d) integer
            out_xyz.append(self.lo + V * self.h)
            out_idx.append(self.index(V))
        return np.concatenate(out_idx), np.concatenate(out_xyz)

    def boundary_facets(self, axis, side):
        """Facets of the Kuhn simplices lying on the face x_axis = lo (side 0) or hi (side 1).

        Returns (nfacet, d) node indices and (nfacet, d, d) coordinates.
        """
        assert not self.periodic
        idx, xyz = self.simplices()
        target = self.lo[axis] if side == 0 else self.hi[axis]
        on = np.isclose(xyz[:, :, axis], target)
        sel = on.sum(axis=1) == self.d
        idx, xyz, on = idx[sel], xyz[sel], on[sel]
        fidx = np.stack([row[m] for row, m in zip(idx, on)]) if len(idx) else np.zeros((0, self.d), np.int64)
        fxyz = np.stack([row[m] for row, m in zip(xyz, on)]) if len(idx) else np.zeros((0, self.d, self.d))
        return fidx, fxyz

    # -- P1 evaluation -------------------------------------------------------
    def eval_lattice_units(self, s):
        """Evaluate all hat functions at points given in lattice units.

        s: (P, d) with s = (x - lo)/h.  Returns (vals (P,n) csr, [grad_a (P,n) csr]).
        """
        s = np.atleast_2d(np.asarray(s, float))
        P = s.shape[0]
        if self.periodic:
            s = np.mod(s, self.ncell)
        cell = np.clip(np.floor(s).astype(np.int64), 0, self.ncell - 1)
        y = s - cell
        perm = np.argsort(-y, axis=1, kind="stable")
        ys = np.take_along_axis(y, perm, axis=1)
        d = self.d
        lam = np.empty((P, d + 1))
        lam[:, 0] = 1.0 - ys[:, 0]
        for k in range(1, d):
            lam[:, k] = ys[:, k - 1] - ys[:, k]
        lam[:, d] = ys[:, d - 1]
        eye = np.eye(d, dtype=np.int64)
        verts = [cell]
        for k in range(d):
            verts.append(verts[-1] + eye[perm[:, k]])
        cols = np.stack([self.index(v) for v in verts], axis=1)           # (P, d+1)
        # gradients in lattice units: d lambda_k / d s
        gl = np.zeros((P, d + 1, d))
        rows = np.arange(P)
        gl[rows, 0, perm[:, 0]] -= 1.0
        for k in range(1, d):
            gl[rows, k, perm[:, k - 1]] += 1.0
            gl[rows, k, perm[:, k]] -= 1.0
        gl[rows, d, perm[:, d - 1]] += 1.0
        rr = np.repeat(rows, d + 1)
        vals = sp.csr_matrix((lam.ravel(), (rr, cols.ravel())), shape=(P, self.n))
        grads = []
        for a in range(d):
            grads.append(sp.csr_matrix(((gl[:, :, a] / self.h[a]).ravel(), (rr, cols.ravel())),
                                       shape=(P, self.n)))
        return vals, grads

    def eval(self, pts):
        return self.eval_lattice_units((np.atleast_2d(pts) - self.lo) / self.h)


def embedding(coarse: Lattice, fine: Lattice):
    """E_{l+1,l}: matrix of the embedding V_l -> V_{l+1} in the nodal bases.

    Column k holds the values of the coarse hat function k at the fine nodes.
    Fine node multi-index i sits at coarse lattice coordinate i/2 (exact in
    binary), so the entries come out exactly 0, 1/2 or 1.
    """
    assert fine.level == coarse.level + 1
    s = fine.node_multi().astype(float) / 2.0
    vals, _ = coarse.eval_lattice_units(s)
    E = vals.tocsr()
    E.eliminate_zeros()
    return E


def embedding_chain(dom_d, lo, hi, periodic, lfine, lcoarse):
    """E_{lfine,lcoarse} = E_{lfine,lfine-1} ... E_{lcoarse+1,lcoarse}."""
    E = sp.identity(Lattice(dom_d, lo, hi, lcoarse, periodic).n, format="csr")
    for l in range(lcoarse, lfine):
        E = embedding(Lattice(dom_d, lo, hi, l, periodic), Lattice(dom_d, lo, hi, l + 1, periodic)) @ E
    return E.tocsr()
