"""Quadrature rules on simplices (collapsed-coordinate Gauss-Legendre, Duffy map).

Used only by the brute-force tier O1.  The collapsed map
x_1 = xi_1, x_2 = xi_2 (1 - xi_1), x_3 = xi_3 (1 - xi_1)(1 - xi_2) turns the unit
cube into the reference simplex with Jacobian prod_j (1 - xi_j)^(k-1-j); a tensor
Gauss rule with n points per direction is then exact for total degree 2n-1-(k-1)
or more.  n = 5 covers every integrand that occurs (degree <= 6 per domain).
"""
from __future__ import annotations

import math

import numpy as np


def _gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def reference_simplex_rule(k, n=5):
    """Points (Q, k) and weights (Q,) on {x >= 0, sum x <= 1}; weights sum to 1/k!."""
    if k == 0:
        return np.zeros((1, 0)), np.ones(1)
    g, gw = _gauss01(n)
    grids = np.meshgrid(*([g] * k), indexing="ij")
    wgrids = np.meshgrid(*([gw] * k), indexing="ij")
    xi = [a.ravel() for a in grids]
    w = np.ones_like(xi[0])
    for a in wgrids:
        w = w * a.ravel()
    pts = np.zeros((xi[0].size, k))
    scale = np.ones_like(xi[0])
    for j in range(k):
        pts[:, j] = xi[j] * scale
        scale = scale * (1.0 - xi[j])
    # Jacobian of the collapsed map: prod_j (1 - xi_j)^(k-1-j)
    jac = np.ones_like(xi[0])
    for j in range(k - 1):
        jac = jac * (1.0 - xi[j]) ** (k - 1 - j)
    return pts, w * jac


def simplex_rule(verts, n=5):
    """Map the reference rule to simplices with vertex coordinates (S, k+1, D).

    Returns points (S*Q, D) and weights (S*Q,).
    """
    S, kp1, D = verts.shape
    k = kp1 - 1
    rp, rw = reference_simplex_rule(k, n)
    lam = np.concatenate([1.0 - rp.sum(axis=1, keepdims=True), rp], axis=1)   # (Q, k+1)
    pts = np.einsum("qi,sid->sqd", lam, verts).reshape(-1, D)
    if k == 0:
        meas = np.ones(S)
    else:
        Ed = verts[:, 1:, :] - verts[:, :1, :]
        G = np.einsum("sid,sjd->sij", Ed, Ed)
        meas = np.sqrt(np.abs(np.linalg.det(G))) / math.factorial(k)
    w = (meas[:, None] * rw[None, :] * math.factorial(k)).reshape(-1)
    return pts, w
