"""GPU parity of the Vlasov-Poisson coupling (Sect. 5.3) through the C ABI:
the density (v-moment plus the prolongation chain), the field of the Poisson
problem, one strip of the fixed point against the oracle's, and the
1+1-dimensional Landau damping rate on the device."""
import math
import sys

import numpy as np
import pytest

from oracle import vlasov as V
from oracle import strip as ostrip
from oracle.operator import Problem
from workloads import random_vector

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


CASES = [(1, 4), (2, 3)]


@pytest.mark.parametrize("d,pl", CASES, ids=[f"d{d}_L{p}" for d, p in CASES])
def test_density_and_field_match_oracle(dev, d, pl):
    from paper_2204_05988_amd import sgdg
    w = V.landau_workload(d=d, paper_level=pl)
    P = Problem(w)
    vp = sgdg.VlasovPoisson(w)
    _say(f"density and field d={d} paper level {pl}: {vp.n_fine} x-nodes, {vp.ndof} DOFs")
    u = random_vector(vp.ndof, 3)[0]
    ut = torch.tensor(u, device=dev)
    for tau in (-1.0, 0.0, 1.0):
        rho = vp.density(ut, P.R, tau).cpu().numpy()
        ref = V.density(P, V.slice_at(P, u, tau))
        e = _rel(rho, ref)
        _say(f"  density at tau={tau}: rel err {e:.2e}")
        assert e <= 1e-12
    u0 = ostrip.initial_coefficients(P)
    rho0 = vp.density(torch.tensor(u0, device=dev), 1)
    rref = V.density(P, u0)
    assert _rel(rho0.cpu().numpy(), rref) <= 1e-12
    E, en = vp.field(rho0)
    Eref, _ = V.poisson_field(w, rref)
    eE = _rel(E.cpu().numpy(), Eref.ravel())
    en_ref = V.electric_energy(w, Eref)
    _say(f"  field rel err {eE:.2e}, energy {en:.6e} (oracle {en_ref:.6e})")
    assert eE <= 1e-9
    assert abs(en - en_ref) <= 1e-9 * en_ref
    vp.close()


@pytest.mark.parametrize("d,pl", CASES, ids=[f"d{d}_L{p}" for d, p in CASES])
def test_fixed_point_strip_matches_oracle(dev, d, pl):
    """Strip 1 of the Landau problem: the device fixed point and the oracle's reach
    the same field and the same density function."""
    from paper_2204_05988_amd import sgdg
    w0 = V.landau_workload(d=d, paper_level=pl)
    P0 = Problem(w0)
    mats = V.field_matrices(w0)
    u0 = ostrip.initial_coefficients(P0)
    E0, _ = V.poisson_field(w0, V.density(P0, u0), mats)
    u_ref, E_ref, its, ch, P = V.vp_strip(d, pl, w0.r, w0.dt, 1, u0, 1, E0, mats, tol=1e-11, fp_tol=1e-10)
    vp = sgdg.VlasovPoisson(w0)
    f, E, st = vp.strip(torch.tensor(u0, device=dev), 1, torch.tensor(E0.ravel(), device=dev), fp_tol=1e-10,
                        solve=sgdg.default_solve_opts(rtol=1e-11, maxit=300))
    _say(f"  d={d}: device {st.fp_iters} fixed-point iterations (oracle {its}), {st.outer_iters} FGMRES, "
         f"dE {st.dE:.1e} df {st.df:.1e}, {st.seconds:.3f}s ({st.assemble_seconds:.3f}s assembly)")
    eE = _rel(E.cpu().numpy(), E_ref.ravel())
    diff = f.cpu().numpy() - u_ref
    dist = 0.0
    for s in range(P.R):
        e1 = np.concatenate([b[s].ravel() for b in P.split(diff)])
        dist += abs(e1 @ P.apply_mass(e1))
    nrm = 0.0
    for s in range(P.R):
        e1 = np.concatenate([b[s].ravel() for b in P.split(u_ref)])
        nrm += abs(e1 @ P.apply_mass(e1))
    dist = math.sqrt(dist / nrm)
    _say(f"  field rel err {eE:.2e}, L2 distance of the densities {dist:.2e}")
    assert eE <= 1e-7
    assert dist <= 1e-8
    vp.close()


@pytest.mark.parametrize("d,pl", CASES, ids=[f"d{d}_L{p}" for d, p in CASES])
def test_strip_on_a_used_handle_equals_a_fresh_one(dev, d, pl):
    """Every fixed-point iteration rewrites the operator's factor tables in place
    for the new field.  A strip run on a handle whose operator has already been
    rewritten for other fields (a strip from another initial state) gives, bit for
    bit, what a new handle gives for the same inputs."""
    from paper_2204_05988_amd import sgdg
    w0 = V.landau_workload(d=d, paper_level=pl)
    P0 = Problem(w0)
    u0 = torch.tensor(ostrip.initial_coefficients(P0), device=dev)
    opts = sgdg.default_solve_opts(rtol=1e-11, maxit=300)
    fresh = sgdg.VlasovPoisson(w0)
    E0, _ = fresh.field(fresh.density(u0, 1))
    fa, Ea, sa = fresh.strip(u0, 1, E0, fp_tol=1e-10, solve=opts)
    fresh.close()
    used = sgdg.VlasovPoisson(w0)
    # another state (twice the perturbation, so other fields) on the same grids
    w1 = V.landau_workload(d=d, paper_level=pl, alpha=2e-2)
    u1 = torch.tensor(ostrip.initial_coefficients(Problem(w1)), device=dev)
    E1, _ = used.field(used.density(u1, 1))
    _, _, s1 = used.strip(u1, 1, E1, fp_tol=1e-10, solve=opts)
    fb, Eb, sb = used.strip(u0, 1, E0, fp_tol=1e-10, solve=opts)
    used.close()
    _say(f"  d={d}: fresh {sa.fp_iters} iterations ({sa.assemble_seconds:.3f}s assembly), "
         f"used handle {s1.fp_iters} + {sb.fp_iters} ({sb.assemble_seconds:.3f}s)")
    assert sa.fp_iters == sb.fp_iters
    assert torch.equal(fa, fb)
    assert torch.equal(Ea, Eb)


def test_landau_damping_on_the_device(dev):
    """36 strips of the 1+1-dimensional Landau problem (paper level 5, 0.5 time
    units per strip) on the device: the field decays at gamma ~ 0.153 and the
    mass is conserved."""
    from paper_2204_05988_amd import sgdg
    w = V.landau_workload(d=1, paper_level=5)
    P = Problem(w)
    vp = sgdg.VlasovPoisson(w)
    f = torch.tensor(ostrip.initial_coefficients(P), device=dev)
    E, en0 = vp.field(vp.density(f, 1))
    prev = 1
    rec = [dict(t=0.0, energy=en0)]
    m0 = V.mass(P, f.cpu().numpy())
    fps = []
    for j in range(1, 37):
        f, Emid, st = vp.strip(f, prev, E, fp_tol=1e-6)
        prev = P.R
        E, en = vp.field(vp.density(f, P.R, 1.0))
        rec.append(dict(t=0.5 * j, energy=en))
        fps.append(st.fp_iters)
    gamma, tp, ep = V.decay_rate(rec)
    m1 = V.mass(P, ostrip.trace_right(P, f.cpu().numpy(), P.R))
    _say(f"  gamma {gamma:.4f}, fixed-point iterations {fps}, mass drift {abs(m1 / m0 - 1):.2e}")
    assert abs(gamma - 0.153) < 0.1 * 0.153
    assert abs(m1 / m0 - 1) < 1e-6
    vp.close()


def test_twostream_instability_grows_at_the_linear_rate(dev):
    """The 1+1-dimensional two-stream instability of Sect. 5.3 (alpha = 1e-3,
    k = 1/5, v0 = 2.4 on (0, 10 pi) x (-9, 9), paper level 5, 0.5 time units per
    strip) on the device: once the growing mode dominates (t in [10, 20]) the
    field amplitude grows at the rate of the linear dispersion relation of two
    Maxwellian beams (gamma = 0.2258) to within 10%, and the mass is conserved."""
    from paper_2204_05988_amd import sgdg
    w = V.twostream_workload(d=1, paper_level=5)
    P = Problem(w)
    vp = sgdg.VlasovPoisson(w)
    f = torch.tensor(ostrip.initial_coefficients(P), device=dev)
    E, en0 = vp.field(vp.density(f, 1))
    rec = [dict(t=0.0, energy=en0)]
    m0 = V.mass(P, f.cpu().numpy())
    opts = sgdg.default_solve_opts(rtol=1e-10, pc=sgdg.default_precond_opts(mass_sweeps=-2))
    prev = 1
    for j in range(1, 41):
        f, _, st = vp.strip(f, prev, E, fp_tol=1e-6, solve=opts)
        prev = P.R
        E, en = vp.field(vp.density(f, P.R, 1.0))
        rec.append(dict(t=0.5 * j, energy=en))
    gamma = V.growth_rate(rec, 10.0, 20.0)
    lin = V.twostream_growth_rate(0.2, 2.4)
    m1 = V.mass(P, ostrip.trace_right(P, f.cpu().numpy(), P.R))
    _say(f"  two-stream: growth rate {gamma:.4f} (linear theory {lin:.4f}), energy {rec[20]['energy']:.2e} -> "
         f"{rec[40]['energy']:.2e}, mass drift {abs(m1 / m0 - 1):.2e}")
    assert abs(gamma / lin - 1) < 0.1
    assert rec[40]["energy"] > 10 * rec[20]["energy"]
    assert abs(m1 / m0 - 1) < 1e-6
    vp.close()

