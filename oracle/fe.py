"""Finite-element factor matrices on one level of one domain (Sect. 4.2, (eq:matrices)).

Each spatial matrix of the paper splits, for separable coefficients, into
d-dimensional factors over Omega^(1) or Omega^(2).  The factor kinds needed are

    mass     M[w]_{k,k'}       = (w phi_k', phi_k)
    deriv    D_a[w]_{k,k'}     = (w d_a phi_k', phi_k)
    stiff    S_ab[w]_{k,k'}    = (w d_a phi_k', d_b phi_k)
    face     F_f[w]_{k,k'}     = integral over the boundary face f of w phi_k' phi_k

with row k = test function and column k' = trial function.  The weight w is a
product of P1 fields (nodal values), so every integrand is a polynomial on each
simplex and is integrated exactly with the barycentric monomial formula
    int_K prod_i lambda_i^{a_i} = d! |K| prod_i a_i! / (d + sum_i a_i)!.

Parity: pinned by the tests (1D closed forms, 1^T M 1 = |Omega|, D 1 = 0,
S 1 = 0, symmetry, agreement with the pointwise-quadrature tier O1).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

from .mesh import Lattice


def _monomial(alpha, dim):
    """int_K prod lambda^alpha / |K| for a dim-simplex K (barycentric formula)."""
    num = 1.0
    for a in alpha:
        num *= math.factorial(a)
    return math.factorial(dim) * num / math.factorial(dim + int(sum(alpha)))


def _weighted_moments(vertex_fields, dim, nverts, extra):
    """int_K w * lambda^(extra multi-index) / |K| for every simplex.

    vertex_fields: list of (nsimp, nverts) nodal values of the weight's factors.
    extra: tuple of vertex indices appended to the monomial (basis functions).
    """
    nsimp = vertex_fields[0].shape[0] if vertex_fields else None
    out = 0.0
    m = len(vertex_fields)
    for tup in itertools.product(range(nverts), repeat=m):
        alpha = [0] * nverts
        for t in tup:
            alpha[t] += 1
        for e in extra:
            alpha[e] += 1
        coef = _monomial(alpha, dim)
        prod = 1.0
        for f, t in zip(vertex_fields, tup):
            prod = prod * f[:, t]
        out = out + coef * prod
    return out


def _bary_gradients(xyz):
    """Gradients of the barycentric coordinates (nsimp, d+1, d) and volumes (nsimp,)."""
    d = xyz.shape[2]
    J = np.transpose(xyz[:, 1:, :] - xyz[:, :1, :], (0, 2, 1))   # (nsimp, d, d): columns = edges
    Jinv = np.linalg.inv(J)
    g = np.empty((xyz.shape[0], d + 1, d))
    g[:, 1:, :] = Jinv                        # row k of J^{-1} = grad lambda_{k+1}
    g[:, 0, :] = -Jinv.sum(axis=1)
    vol = np.abs(np.linalg.det(J)) / math.factorial(d)
    return g, vol


def _facet_measure(xyz):
    """(d-1)-dimensional measure of facets given by (nf, d, d) vertex coordinates."""
    nf, nv, d = xyz.shape
    if nv == 1:
        return np.ones(nf)
    E = xyz[:, 1:, :] - xyz[:, :1, :]           # (nf, d-1, d)
    G = np.einsum("fid,fjd->fij", E, E)
    return np.sqrt(np.abs(np.linalg.det(G))) / math.factorial(nv - 1)


def weight_nodal(fields_by_name, spec, n):
    """Nodal values of a weight spec (scale, field_names, kink) on the finest lattice.

    kink None: scale * prod fields.  'pos': max(that, 0).  'neg': max(-that, 0).
    Returns a list of nodal factor arrays (the product's factors) and a scale.
    A kinked weight is the P1 interpolant of the kinked product (one field).
    """
    scale, names, kink = spec
    if kink is None:
        return float(scale), [fields_by_name[k] for k in names]
    prod = np.full(n, float(scale))
    for k in names:
        prod = prod * fields_by_name[k]
    if kink == "pos":
        return 1.0, [np.maximum(prod, 0.0)]
    if kink == "neg":
        return 1.0, [np.maximum(-prod, 0.0)]
    raise ValueError(kink)


def assemble(lat: Lattice, kind, weight_fields, scale=1.0, a=None, b=None, face=None):
    """Assemble one factor matrix on lattice `lat` (rows test, columns trial)."""
    d = lat.d
    if kind == "face":
        axis, side = face
        fidx, fxyz = lat.boundary_facets(axis, side)
        meas = _facet_measure(fxyz)
        vf = [w[fidx] for w in weight_fields]
        nv = d
        rows, cols, vals = [], [], []
        for p in range(nv):
            for q in range(nv):
                mom = _weighted_moments(vf, d - 1, nv, (p, q))
                rows.append(fidx[:, p]); cols.append(fidx[:, q])
                vals.append(scale * meas * mom * np.ones(len(fidx)))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(lat.n, lat.n))
    idx, xyz = lat.simplices()
    grad, vol = _bary_gradients(xyz)
    vf = [w[idx] for w in weight_fields]
    nv = d + 1
    rows, cols, vals = [], [], []
    if kind == "mass":
        for p in range(nv):
            for q in range(nv):
                mom = _weighted_moments(vf, d, nv, (p, q))
                rows.append(idx[:, p]); cols.append(idx[:, q])
                vals.append(scale * vol * mom * np.ones(len(idx)))
    elif kind == "deriv":
        for p in range(nv):                  # test
            mom = _weighted_moments(vf, d, nv, (p,))
            for q in range(nv):              # trial
                rows.append(idx[:, p]); cols.append(idx[:, q])
                vals.append(scale * vol * mom * grad[:, q, a])
    elif kind == "stiff":
        mom = _weighted_moments(vf, d, nv, ())
        for p in range(nv):
            for q in range(nv):
                rows.append(idx[:, p]); cols.append(idx[:, q])
                vals.append(scale * vol * mom * grad[:, q, a] * grad[:, p, b])
    else:
        raise ValueError(kind)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(lat.n, lat.n))
