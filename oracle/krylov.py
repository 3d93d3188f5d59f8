"""Flexible GMRES (right preconditioned), FP64, the outer solver of each strip.

The paper wraps the combination-technique preconditioner in a Richardson
iteration (Algorithm 1).  The workloads here ask for a Krylov outer solve to a
relative residual; flexible GMRES with the same preconditioner is used, which
minimises ||b - A u||_2 over the preconditioned Krylov space.  Arnoldi uses
classical Gram-Schmidt applied twice; the small least-squares problem uses
Givens rotations.  The stopping test is the true relative residual
||b - A u|| / ||b|| <= tol, checked at the end of every restart cycle and
whenever the Arnoldi estimate drops below tol.

Parity: pinned by the tests (exact solve of small nonsingular systems; with
P = A^{-1} it converges in one iteration).
"""
from __future__ import annotations

import numpy as np


def fgmres(apply_A, b, precond=None, x0=None, tol=1e-10, restart=50, maxit=500, callback=None):
    b = np.asarray(b, float)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, float)
    precond = precond or (lambda v: v)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, dict(iters=0, rel=0.0, history=[0.0])
    total = 0
    history = []
    r = b - apply_A(x)
    beta = np.linalg.norm(r)
    history.append(beta / bnorm)
    while total < maxit and beta / bnorm > tol:
        m = min(restart, maxit - total)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m); sn = np.zeros(m)
        g = np.zeros(m + 1); g[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = apply_A(Z[j])
            for _ in range(2):                      # CGS2
                h = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h
                H[:j + 1, j] += h
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            if hnext > 0:
                V[j + 1] = w / hnext
            for i in range(j):                      # apply previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den; H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]; g[j] = cs[j] * g[j]
            total += 1
            k_used = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if callback:
                callback(total, abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or hnext == 0.0:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + Z[:k_used].T @ y
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if k_used == 0:
            break
    return x, dict(iters=total, rel=beta / bnorm, history=history)
