"""Pins of the Vlasov-Poisson oracle (Sect. 5.3): the density, the field of the
Poisson problem and the coupled fixed point, against facts fixed by the
mathematics and by linear theory (Landau damping)."""
import math

import numpy as np
import pytest

from workloads import lattice_coords
from oracle import vlasov as V
from oracle.operator import Problem


def test_density_of_a_single_grid_product_is_exact():
    """f = g(x) h(v) on one component grid: rho = g * int h dv, the v-integral of a P1
    function being the trapezoidal sum on its lattice."""
    w = V.landau_workload(d=1, paper_level=3)
    P = Problem(w)
    rng = np.random.default_rng(2)
    u = np.zeros(P.ndof // P.R)
    off = 0
    for gi, (lx, lv) in enumerate(P.upper):
        n = P.nx(lx) * P.nv(lv)
        if gi == 1:
            g = rng.standard_normal(P.nx(lx))
            h = rng.standard_normal(P.nv(lv))
            u[off:off + n] = np.outer(g, h).ravel()
            X = lattice_coords(w.v, lv)[:, 0]
            integral = float(np.sum(0.5 * (h[1:] + h[:-1]) * np.diff(X)))
            gl, lxg = g, lx
        off += n
    rho = V.density(P, u)
    ref = P.E("x", w.L, lxg) @ gl * integral
    assert np.abs(rho - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("d", [1, 2])
def test_poisson_field_converges_at_second_order(d):
    """rho = 1 + a sum_i cos(k x_i) gives E_i = -(a/k) sin(k x_i) exactly; the P1 field
    (L2 projection of -grad phi) converges at second order in the nodal max norm."""
    a, k = 0.3, 0.5
    errs = []
    for pl in (3, 4, 5):
        w = V.landau_workload(d=d, paper_level=pl)
        X = lattice_coords(w.x, w.L)
        rho = 1 + a * np.sum(np.cos(k * X), axis=1)
        E, phi = V.poisson_field(w, rho)
        ref = -(a / k) * np.sin(k * X).T
        errs.append(np.abs(E - ref).max())
        assert abs(np.mean(phi)) < 1e-12
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)


def test_landau_damping_rate():
    """1+1-dimensional Landau damping (alpha = 0.01, k = 1/2, v in (-6, 6)) at the
    paper's level 5 with 0.5 time units per strip: the electric energy oscillates at
    twice the plasma frequency (omega ~ 1.4156 from linear theory, peaks pi/omega
    apart) and its peaks decay as exp(-2 gamma t) with gamma ~ 0.153; the fixed
    point conserves the mass to the solver tolerance."""
    rec = V.landau_run(d=1, paper_level=5, r=1, dt=0.5, nstrips=36, fp_tol=1e-6)
    gamma, tp, ep = V.decay_rate(rec)
    spacing = float(np.mean(np.diff(tp)))
    omega = math.pi / spacing
    drift = abs(rec[-1]["mass"] / rec[0]["mass"] - 1)
    assert abs(gamma - 0.153) < 0.1 * 0.153, gamma
    assert abs(omega - 1.4156) < 0.1 * 1.4156, omega
    assert drift < 1e-6, drift
    assert rec[-1]["energy"] < 0.01 * rec[0]["energy"]


def test_landau_root_damps_at_the_papers_rate():
    """The least-damped root of a unit Maxwellian's dielectric function at k = 1/2
    damps at the rate the paper quotes from linear analysis (gamma ~ 0.153)."""
    w = V.landau_mode(0.5)
    assert abs(V.dielectric(w, 0.5, [(1.0, 0.0, 1.0)])) < 1e-12
    assert abs(-w.imag - 0.153) < 0.0006
    assert 1.40 < w.real < 1.43


def test_twostream_rate_tends_to_cold_beams():
    """As the thermal speed goes to zero the two-stream growth rate tends to the
    closed form of two cold beams; at unit thermal speed it is smaller."""
    cold = V.cold_twostream_growth_rate(0.2, 2.4)
    a, om = 0.2 * 2.4, 1j * cold
    assert abs(0.5 * (1 / (om - a) ** 2 + 1 / (om + a) ** 2) - 1) < 1e-12  # the cold beams' dispersion relation
    for vth, tol in ((1e-2, 1e-4), (1e-3, 1e-6)):
        assert abs(V.twostream_growth_rate(0.2, 2.4, vth) - cold) < tol
    g = V.twostream_growth_rate(0.2, 2.4, 1.0)
    assert 0.0 < g < cold
    beams = [(0.5, 2.4, 1.0), (0.5, -2.4, 1.0)]
    assert abs(V.dielectric(1j * g, 0.2, beams)) < 1e-10
    for s in (0.1, 0.3, 1.0):
        assert abs(V.dielectric(1j * s, 0.2, beams).imag) < 1e-12
    # a single beam (no counter-stream) is stable
    assert V.twostream_growth_rate(0.2, 0.0, 1.0) == 0.0

