"""GPU parity for coefficients that depend on time (Sect. 4.2, the block formula
with an m-point time quadrature), through the C ABI: the operators of a strip
whose coefficients move in time against the oracle's quadrature form, the
right-hand side, and strip solves that must reproduce a discrete exact solution
and reach the tolerance under the oracle's time-dependent operator."""
import sys

import numpy as np
import pytest

from workloads import config_c4_member, config_timedep_exact, gauss_legendre_times, random_vector, sample_on_grids
from oracle.ct import CTPreconditioner
from oracle.krylov import fgmres
from oracle.operator import Problem
from oracle import strip as ostrip

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_05988_amd import sgdg
    sgdg.lib()
    return torch.device("cuda:0")


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = {
    "exact_d1": lambda: config_timedep_exact(1, 1, 4),
    "exact_d2": lambda: config_timedep_exact(2, 1, 2),
    "c4t_L5": lambda: config_c4_member(3, L=5, tvary=1.0),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("kind", [0, 1, 3, 4], ids=["full", "blockdiag", "data_f", "data_g"])
def test_time_dependent_apply(dev, case, kind):
    from paper_2204_05988_amd import sgdg
    w = CASES[case]()
    t0 = 2 * w.dt
    P = Problem(w, t0=t0)
    ops = sgdg.SparseGridOps(w, t0=t0)
    u = random_vector(P.ndof, 23)[0]
    if kind == 0:
        ref = P.apply(u)
    elif kind == 3:
        ref = P.apply(u, P.data_terms())
    elif kind == 4:
        terms = P.inflow_data_terms()
        ref = P.apply(u, terms) if terms else np.zeros_like(u)
    else:
        ref = np.concatenate([P.block_apply(P.terms, l, l, ub).ravel() for l, ub in zip(P.upper, P.split(u))])
    _say(f"time-dependent apply {case} kind {kind}: {P.ndof} DOFs, {ops.op_info(kind)['nterms']} terms")
    ut = torch.tensor(u, device=dev)
    y = torch.empty_like(ut)
    ops.apply(ut, y, kind)
    y32 = torch.empty(P.ndof, dtype=torch.float32, device=dev)
    ops.apply(ut.float(), y32, kind)
    torch.cuda.synchronize()
    if np.abs(ref).max() == 0:
        assert np.abs(y.cpu().numpy()).max() == 0
        return
    e64, e32 = _rel(y.cpu().numpy(), ref), _rel(y32.double().cpu().numpy(), ref)
    _say(f"  fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= 1e-10 and e32 <= 2e-5
    ops.close()


def _nodal(w, P, fn, j):
    tq, _ = gauss_legendre_times((j - 1) * w.dt, w.dt, w.r + 2)
    return np.stack([np.concatenate([sample_on_grids(w, P.upper, fn, t), sample_on_grids(w, P.lower, fn, t)])
                     for t in tq])


@pytest.mark.parametrize("d,L", [(1, 4), (2, 2)])
def test_time_dependent_exact_solution_on_the_device(dev, d, L):
    """Two strips of the discrete-exact problem entirely on the device (rhs with its own
    f and g, solve): each strip returns u, measured with the oracle's mass."""
    from paper_2204_05988_amd import sgdg
    w = config_timedep_exact(d, 1, L)
    P1 = Problem(w)
    u_prev = torch.tensor(ostrip.initial_coefficients(P1), device=dev)
    prev = 1
    for j in (1, 2):
        t0 = (j - 1) * w.dt
        P = Problem(w, t0=t0)
        ops = sgdg.SparseGridOps(w, t0=t0)
        b = ops.rhs(u_prev, prev, torch.tensor(_nodal(w, P, w.f, j), device=dev),
                    torch.tensor(_nodal(w, P, w.g, j), device=dev))
        b_ref = ostrip.rhs(P, j, u_prev.cpu().numpy(), prev)
        assert _rel(b.cpu().numpy(), b_ref) <= 1e-10
        x, st = ops.solve_strip(b, torch.zeros_like(b), sgdg.default_solve_opts(rtol=1e-12, maxit=300))
        xs = x.cpu().numpy()
        tq = np.cos(np.pi * (np.arange(P.R) + 0.5) / P.R)
        Vd = np.linalg.inv(np.polynomial.legendre.legvander(tq, P.R - 1))
        vals = [ostrip.interpolate(P, lambda X, V, t=t0 + 0.5 * w.dt * (tk + 1): w.exact(t, X, V)) for tk in tq]
        ref = [sum(Vd[s, k] * vals[k] for k in range(P.R)) for s in range(P.R)]
        err2 = ref2 = 0.0
        for s in range(P.R):
            us = np.concatenate([bb[s].ravel() for bb in P.split(xs)])
            e = us - ref[s]
            err2 += abs(e @ P.apply_mass(e))
            ref2 += abs(ref[s] @ P.apply_mass(ref[s]))
        _say(f"  d={d} strip {j}: {st.outer_iters} iterations, L2 error to the exact solution "
             f"{np.sqrt(err2 / ref2):.2e}")
        assert np.sqrt(err2 / ref2) <= 1e-9
        u_prev, prev = x, P.R
        ops.close()


def test_time_dependent_strip_solve(dev):
    """A strip of the 4D problem with moving coefficients (FP64 and mixed precision)
    reaches 1e-8 under the oracle's time-dependent operator."""
    from paper_2204_05988_amd import sgdg
    w = config_c4_member(3, L=5, tvary=1.0)
    t0 = w.dt
    P = Problem(w, t0=t0)
    ops = sgdg.SparseGridOps(w, t0=t0)
    b_ref = P.apply(random_vector(P.ndof, 8)[0])
    b = torch.tensor(b_ref, device=dev)
    for mixed in (False, True):
        x, st = ops.solve_strip(b, torch.zeros_like(b), sgdg.default_solve_opts(rtol=1e-8, mixed=mixed))
        res = np.linalg.norm(b_ref - P.apply(x.cpu().numpy())) / np.linalg.norm(b_ref)
        _say(f"  {'mixed' if mixed else 'fp64'}: {st.outer_iters} iterations, oracle residual {res:.2e}")
        assert res <= 1e-8 * (1 + 1e-6)
    ops.close()
