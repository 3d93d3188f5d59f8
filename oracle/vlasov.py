"""Vlasov-Poisson by a fixed-point iteration per time strip (Sect. 5.3).
Test infrastructure: a plain CPU FP64 reference, not part of the product path.

The electron density f(t, x, v) in a neutralising ion background obeys the
transport equation (eq:transport) with the field-dependent velocity
beta = (v, -E(x)) coupled to the Poisson problem (eq:poisson)

    -Laplace_x phi = 1 - rho,   rho(x) = int f(x, v) dv,   E = -grad_x phi.

Per strip I_j the two are solved alternately (eq:E_f): start from the field of
f(t_{j-1}^-); solve the linear transport with that field for f^(k+1); take the
density of f^(k+1) at the strip's midpoint (the midpoint rule of Sect. 5.3, so
the field is constant over the strip); solve the Poisson problem for the new
field; stop when the field and the density function change by less than a
tolerance.

Discrete readings (the paper names the method only):
  * rho is the v-integral of the sparse-grid function, grid by grid:
    rho_l(x) = sum_{kx} (sum_{kv} u_l[kx, kv] int phi_kv dv) phi_kx(x), a P1
    function on x-level lx, prolongated to the finest x-lattice and summed;
  * the Poisson problem is solved with P1 elements on the finest x-lattice,
    K phi = M (1 - rho), phi of mean zero (the x-domain is periodic);
  * E_i is the L2 projection of -d_i phi onto P1: M E_i = -D_i phi, with
    D_i[k, k'] = (d_i phi_k', phi_k);
  * the change of f is measured in L2 (cross-grid mass), the paper's H1 norm
    being a stopping heuristic.

The linear theory at the end (the dielectric function of Maxwellian beams and
its roots) is an independent check of the runs' rates, not part of the scheme.

Parity: pinned by the tests -- a density of a single-grid product function
integrates exactly; the discrete field of rho = 1 + a cos(k x) converges to
-(a/k) sin(k x) at second order; the 1+1-dimensional Landau damping decays at
the linear-theory rate gamma ~ 0.153 with mass conserved to the solver
tolerance; the dielectric root of a Maxwellian at k = 1/2 damps at the
paper's 0.153, the two-stream rate tends to the closed form of cold beams as
the thermal speed goes to zero, and the symmetric two-stream dielectric is real
on the imaginary axis.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import config_landau, config_twostream

from .ct import CTPreconditioner
from .fe import assemble
from .krylov import fgmres
from .mesh import Lattice
from .operator import Problem, _fkey
from . import strip as ostrip
from .timedg import eta


def landau_workload(d=1, paper_level=5, r=1, dt=0.5, alpha=1e-2, k=0.5, E=None, vmax=6.0):
    """The Landau-damping workload (its data live with the other workloads)."""
    return config_landau(d, paper_level, r, dt, alpha, k, E, vmax)


def slice_at(P, u, tau):
    """Coefficients of the strip function at reference time tau in [-1, 1] (one slice)."""
    R = P.R
    w = np.array([eta(s, tau) for s in range(R)])
    out, off = [], 0
    for (lx, lv) in P.upper:
        n = P.nx(lx) * P.nv(lv)
        out.append(w @ u[off:off + R * n].reshape(R, n))
        off += R * n
    return np.concatenate(out)


def density(P, u1):
    """rho on the finest x-lattice of a one-slice sparse-grid function."""
    L = P.w.L
    rho = np.zeros(P.nx(L))
    off = 0
    for (lx, lv) in P.upper:
        n = P.nx(lx) * P.nv(lv)
        U = u1[off:off + n].reshape(P.nx(lx), P.nv(lv))
        mv = P.factor("v", _fkey("mass"), lv, lv) @ np.ones(P.nv(lv))      # int phi_kv dv
        rho += P.E("x", L, lx) @ (U @ mv)
        off += n
    return rho


def field_matrices(w):
    """Finest-level x matrices: stiffness sum_i S_ii, mass M and derivatives D_i."""
    lat = Lattice(w.x.d, w.x.lo, w.x.hi, w.L, w.x.periodic)
    K = sum(assemble(lat, "stiff", [], a=i, b=i) for i in range(w.x.d)).tocsr()
    M = assemble(lat, "mass", []).tocsr()
    D = [assemble(lat, "deriv", [], a=i).tocsr() for i in range(w.x.d)]
    return K, M, D


def poisson_field(w, rho, mats=None):
    """E (shape [d][n]) and phi from K phi = M (1 - rho), mean(phi) = 0, M E_i = -D_i phi."""
    K, M, D = mats or field_matrices(w)
    n = K.shape[0]
    rhs = M @ (1.0 - rho)
    one = np.ones((n, 1))
    Kb = sp.bmat([[K, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc()
    sol = spla.spsolve(Kb, np.concatenate([rhs, [0.0]]))
    phi = sol[:n]
    Mlu = spla.splu(M.tocsc())
    E = np.stack([-Mlu.solve(Di @ phi) for Di in D])
    return E, phi


def electric_energy(w, E, mats=None):
    K, M, D = mats or field_matrices(w)
    return 0.5 * sum(float(Ei @ (M @ Ei)) for Ei in E)


def mass(P, u1):
    """int f dx dv: the cross-grid mass product tested with the constant 1 of one
    grid (the first upper grid; every grid's space holds the constants)."""
    n = P.nx(P.upper[0][0]) * P.nv(P.upper[0][1])
    return float(np.sum(P.apply_mass(u1)[:n]))


def vp_strip(d, paper_level, r, dt, j, u_prev, R_prev, E0, mats, tol=1e-8, fp_tol=1e-9, max_fp=20, **kw):
    """One strip of the fixed point: returns (u, E, fixed-point iterations, last changes)."""
    E = E0
    u_old = None
    for it in range(1, max_fp + 1):
        w = landau_workload(d, paper_level, r, dt, E=E, **kw)
        P = Problem(w)
        b = ostrip.rhs(P, j, u_prev, R_prev)
        u, _ = fgmres(P.apply, b, CTPreconditioner(P), tol=tol, restart=50, maxit=300)
        rho = density(P, slice_at(P, u, 0.0))
        E_new, _ = poisson_field(w, rho, mats)
        dE = float(np.abs(E_new - E).max())
        if u_old is None:
            du = float("inf")
        else:
            e = slice_at(P, u - u_old, 0.0)
            du = math.sqrt(abs(e @ P.apply_mass(e)))
        E, u_old = E_new, u
        if dE + du < fp_tol:
            break
    return u, E, it, (dE, du), P


def landau_run(d=1, paper_level=5, r=1, dt=0.5, nstrips=30, tol=1e-8, fp_tol=1e-9, **kw):
    """March the fixed point strip by strip; returns per-strip-end records."""
    w0 = landau_workload(d, paper_level, r, dt, **kw)
    mats = field_matrices(w0)
    P0 = Problem(w0)
    u_prev = ostrip.initial_coefficients(P0)
    R_prev = 1
    E, _ = poisson_field(w0, density(P0, u_prev), mats)
    rec = [dict(t=0.0, energy=electric_energy(w0, E, mats), mass=mass(P0, u_prev), iters=0)]
    for j in range(1, nstrips + 1):
        u, E_mid, its, ch, P = vp_strip(d, paper_level, r, dt, j, u_prev, R_prev, E, mats, tol=tol,
                                        fp_tol=fp_tol, **kw)
        tr = ostrip.trace_right(P, u, P.R)
        E, _ = poisson_field(w0, density(P, tr), mats)
        rec.append(dict(t=j * dt, energy=electric_energy(w0, E, mats), mass=mass(P, tr), iters=its,
                        dE=ch[0], du=ch[1]))
        u_prev, R_prev = u, P.R
    return rec


def decay_rate(rec, t_max=None):
    """Damping rate of the field amplitude from the local maxima of the electric
    energy (energy ~ exp(-2 gamma t)): least-squares slope of log(peaks) / -2."""
    t = np.array([r["t"] for r in rec])
    e = np.array([r["energy"] for r in rec])
    keep = np.ones_like(t, bool) if t_max is None else t <= t_max
    t, e = t[keep], e[keep]
    pk = [i for i in range(1, len(e) - 1) if e[i] >= e[i - 1] and e[i] >= e[i + 1]]
    slope = np.polyfit(t[pk], np.log(e[pk]), 1)[0]
    return -0.5 * slope, t[pk], e[pk]


# --- linear theory: an independent check of the runs (not part of the scheme) -------------

def dielectric(omega, k, beams):
    """Longitudinal dielectric function of a plasma of Maxwellian beams, each given
    as (weight, drift u, thermal speed s), in the units of the runs (plasma
    frequency 1):

        eps(omega, k) = 1 + sum_b weight_b (1 + zeta_b Z(zeta_b)) / (k s_b)^2,
        zeta_b = (omega / k - u_b) / (sqrt(2) s_b),

    with the plasma dispersion function Z(zeta) = i sqrt(pi) w(zeta), w the
    Faddeeva function (scipy.special.wofz), which continues the Landau contour
    below the real axis.  Roots in omega are the linear modes exp(i(kx - omega t))."""
    from scipy.special import wofz
    omega = complex(omega)
    out = 1.0 + 0.0j
    for wt, u, sd in beams:
        z = (omega / k - u) / (math.sqrt(2.0) * sd)
        out += wt * (1.0 + z * 1j * math.sqrt(math.pi) * wofz(z)) / (k * sd) ** 2
    return out


def dispersion_root(k, beams, guess, tol=1e-13, maxit=100):
    """A root of eps(., k) = 0 near guess by the secant method."""
    w0, w1 = complex(guess), complex(guess) * (1 + 1e-4) + 1e-6
    f0, f1 = dielectric(w0, k, beams), dielectric(w1, k, beams)
    for _ in range(maxit):
        w2 = w1 - f1 * (w1 - w0) / (f1 - f0)
        if abs(w2 - w1) < tol * max(1.0, abs(w2)):
            return w2
        w0, f0, w1, f1 = w1, f1, w2, dielectric(w2, k, beams)
    raise RuntimeError("dispersion root did not converge")


def landau_mode(k=0.5):
    """Frequency and damping of the least-damped mode of a unit Maxwellian."""
    return dispersion_root(k, [(1.0, 0.0, 1.0)], 1.0 + 1.5 * k * k - 0.1j)


def twostream_growth_rate(k=0.2, v0=2.4, vth=1.0):
    """Growth rate gamma of the symmetric two-stream mode (omega = i gamma) of two
    beams of half the density at +-v0 with thermal speed vth (the field amplitude
    grows as exp(gamma t)); 0 if the mode is stable."""
    from scipy.optimize import brentq
    beams = [(0.5, v0, vth), (0.5, -v0, vth)]
    f = lambda g: dielectric(1j * g, k, beams).real
    hi = k * v0 + 1.0
    if f(1e-9) * f(hi) > 0:
        return 0.0
    return brentq(f, 1e-9, hi, xtol=1e-14)


def cold_twostream_growth_rate(k=0.2, v0=2.4):
    """The cold-beam limit: 1 = (1/2) [1 / (omega - k v0)^2 + 1 / (omega + k v0)^2]
    gives omega^2 = ((2a^2 + 1) - sqrt(8a^2 + 1)) / 2 with a = k v0."""
    a = k * v0
    w2 = ((2 * a * a + 1) - math.sqrt(8 * a * a + 1)) / 2
    return math.sqrt(-w2) if w2 < 0 else 0.0


def growth_rate(rec, t0, t1):
    """Growth rate of the field amplitude from the electric energy records
    (energy ~ exp(2 gamma t)): least-squares slope of log(energy) on [t0, t1] / 2."""
    t = np.array([r["t"] for r in rec])
    e = np.array([r["energy"] for r in rec])
    keep = (t >= t0) & (t <= t1)
    return 0.5 * float(np.polyfit(t[keep], np.log(e[keep]), 1)[0])


def twostream_workload(d=1, paper_level=5, r=1, dt=0.5, **kw):
    """The two-stream workload (its data live with the other workloads)."""
    return config_twostream(d, paper_level, r, dt, **kw)

