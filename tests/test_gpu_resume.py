"""Strip-wise stepping as a checkpoint (Sect. 2: every strip starts from the
previous strip's trace only): a march stopped after strip 3, its coefficients
copied to the host and fed to a fresh handle, continues bit for bit as the
uninterrupted march, and the same march run twice gives the same bits (the
solver's reductions are deterministic)."""
import sys

import numpy as np
import pytest

from workloads import config_c1, config_c2, gauss_legendre_times, sample_on_grids

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


def _grids(shapes):
    return [(lx, lv) for lx, lv, _, _ in shapes]


def _rhs(ops, w, j, u_prev, prev, dev):
    tq, _ = gauss_legendre_times((j - 1) * w.dt, w.dt, w.r + 2)

    def nodal(fn):
        if fn is None:
            return None
        rows = [np.concatenate([sample_on_grids(w, _grids(ops.upper), fn, t),
                                sample_on_grids(w, _grids(ops.lower), fn, t)]) for t in tq]
        return torch.tensor(np.stack(rows), device=dev)

    return ops.rhs(u_prev, prev, nodal(w.f), nodal(w.g))


def _initial(ops, w, dev):
    nodal = np.concatenate([sample_on_grids(w, _grids(ops.upper), w.u0), sample_on_grids(w, _grids(ops.lower), w.u0)])
    u0 = torch.empty(ops.npts_up, dtype=torch.float64, device=dev)
    ops.combine(torch.tensor(nodal, device=dev), u0, 1)
    return u0


def _march(ops, w, u_prev, prev, j0, j1, dev, opts):
    for j in range(j0, j1 + 1):
        b = _rhs(ops, w, j, u_prev, prev, dev)
        u = torch.zeros_like(b)
        ops.solve_strip(b, u, opts)
        u_prev, prev = u, ops.R
    torch.cuda.synchronize()
    return u_prev


@pytest.mark.parametrize("name,fn,strips", [("c1", config_c1, 6), ("c2_L5", lambda: config_c2(L=5), 4)])
def test_march_resumes_bit_identically(dev, name, fn, strips):
    from paper_2204_05988_amd import sgdg
    w = fn()
    opts = sgdg.default_solve_opts(rtol=1e-10, maxit=400)
    ops = sgdg.SparseGridOps(w)
    u0 = _initial(ops, w, dev)
    full = _march(ops, w, u0, 1, 1, strips, dev, opts)
    again = _march(ops, w, u0, 1, 1, strips, dev, opts)
    half = strips // 2
    mid = _march(ops, w, u0, 1, 1, half, dev, opts).cpu().numpy()
    ops.close()
    _say(f"{name}: {strips} strips, checkpoint after strip {half}")
    ops2 = sgdg.SparseGridOps(w)
    resumed = _march(ops2, w, torch.tensor(mid, device=dev), ops2.R, half + 1, strips, dev, opts)
    ops2.close()
    assert torch.equal(full, again)
    assert torch.equal(full, resumed)
