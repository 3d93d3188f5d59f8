"""Discontinuous polynomials in time on one strip I_j (Sect. 2 and Sect. 4.2).

Basis: Legendre polynomials mapped to the strip, eta_s(t) = P_s(2 (t - t_{j-1})/dt - 1),
s = 0..r.  With time-independent coefficients the quadrature sums of Sect. 4.2
become exact integrals:
    Mt[s,s'] = int eta_s' eta_s,   Tt[s,s'] = int eta_s'' eta_s  (eta' = time derivative),
    Ct[s,s'] = int eta_s'' eta_s',  Gt[s,s'] = eta_s'(t_{j-1}) eta_s(t_{j-1}).
They are computed here by Gauss-Legendre quadrature with r+2 points (exact).

Parity: pinned by the tests (closed forms for r=0,1; the (r, r+1) Pade
approximant of exp(-z) for the pure-reaction strip map).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def eta(s, tau):
    """Value of eta_s at reference coordinate tau in [-1, 1]."""
    c = np.zeros(s + 1); c[s] = 1.0
    return npleg.legval(tau, c)


def deta(s, tau, dt):
    """Time derivative of eta_s at reference coordinate tau (chain rule 2/dt)."""
    c = np.zeros(s + 1); c[s] = 1.0
    return npleg.legval(tau, npleg.legder(c)) * (2.0 / dt)


def time_matrices(r, dt):
    R = r + 1
    xg, wg = npleg.leggauss(r + 2)
    w = wg * dt / 2.0
    E = np.array([eta(s, xg) for s in range(R)])          # (R, nq)
    Dd = np.array([deta(s, xg, dt) for s in range(R)])
    Mt = (E * w) @ E.T
    Tt = (E * w) @ Dd.T            # row s (test eta_s), column s' (trial derivative)
    Ct = (Dd * w) @ Dd.T
    left = np.array([eta(s, -1.0) for s in range(R)])
    Gt = np.outer(left, left)
    return Mt, Tt, Ct, Gt


def left_values(r):
    return np.array([eta(s, -1.0) for s in range(r + 1)])


def right_values(r):
    return np.array([eta(s, 1.0) for s in range(r + 1)])


def time_quadrature(r, dt, m):
    """Per-point time matrices of an m-point Gauss-Legendre rule on the strip (Sect. 4.2):
    M_mu = w_mu eta_s'(tau_mu) eta_s(tau_mu), T_mu = w_mu eta'_s'(tau_mu) eta_s(tau_mu),
    C_mu = w_mu eta'_s'(tau_mu) eta'_s(tau_mu) (row s test, column s' trial), with the
    physical weights w_mu (summing to dt) folded in; tau in [-1, 1]."""
    R = r + 1
    xg, wg = npleg.leggauss(m)
    w = wg * dt / 2.0
    E = np.array([eta(s, xg) for s in range(R)])          # (R, m)
    Dd = np.array([deta(s, xg, dt) for s in range(R)])
    M = [w[q] * np.outer(E[:, q], E[:, q]) for q in range(m)]
    T = [w[q] * np.outer(E[:, q], Dd[:, q]) for q in range(m)]
    C = [w[q] * np.outer(Dd[:, q], Dd[:, q]) for q in range(m)]
    return dict(tau=xg, weights=wg, M=M, T=T, C=C)
