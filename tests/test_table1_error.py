"""The SD-norm error of the periodic advection test (Sect. 5.1, Table 1) from
operator applications: the benchmark's evaluator, run here on the oracle's
operators and strip solutions, against the oracle's quadrature of the norm
(eq:norm_SD) on the finest product mesh, and the hat's Fourier coefficient
against the closed form of the 1D hat."""
import numpy as np
import pytest

import bench
from oracle import strip
from oracle.norms import sd_error_periodic
from oracle.operator import Problem
from workloads import config_table1


@pytest.mark.parametrize("level", [2, 3, 6])
def test_hat_fourier_1d_closed_form(level):
    # the 1D hat of width 2h: h (sin(pi h) / (pi h))^2
    h = 2.0 ** -level
    a = bench.hat_fourier(1, level)
    assert abs(a - h * (np.sin(np.pi * h) / (np.pi * h)) ** 2) <= 1e-15
    assert abs(a.imag) <= 1e-17


@pytest.mark.parametrize("d", [2, 3])
def test_hat_fourier_tends_to_the_hat_integral(d):
    # exp(2 pi i sum y) -> 1 as the lattice refines: a_l / h^d -> 1 (the hat integrates to h^d),
    # with the second-order term of a symmetric support
    e = [abs(bench.hat_fourier(d, l) / 2.0 ** (-d * l) - 1) for l in (4, 5, 6)]
    assert e[0] < 0.1 and 3.8 < e[0] / e[1] < 4.2 and 3.8 < e[1] / e[2] < 4.2


@pytest.mark.parametrize("d,Lp", [(1, 2), (1, 3), (2, 1)])
def test_operator_form_equals_quadrature_form(d, Lp):
    w = config_table1(Lp, d=d)
    P = Problem(w)
    sols, st = strip.march(P, tol=1e-12)
    assert all(s["rel"] <= 1e-12 for s in st)
    ref = sd_error_periodic(P, None, sols, w.exact)
    grids = [(lx, lv, P.nx(lx), P.nv(lv)) for lx, lv in P.upper]
    err, parts = bench.sd_error_table1(w, grids, sols, P.apply, P.apply_mass, np.dot, np.concatenate, lambda v: v)
    # the oracle integrates the end terms with the exact solution by a 5-point rule
    assert abs(err / ref - 1) <= 1e-7, (err, ref)
    assert parts["strip"] > 0 and parts["jump"] > 0 and parts["end"] > 0
