"""Properties of the HIP operator at the benchmark sizes, where the oracle's
explicit operator is too large to form, plus degenerate cases.

* constants: the constant function lies in every component space, so the
  per-grid sums of A u (one per time slice) agree for every u (Sect. 4.1:
  the spanning set is redundant; the test function 1 is shared);
* kernel vectors: c on the lower grid (lx, lv-1), prolonged in v onto upper
  grid (lx, lv) and, with the opposite sign, in x onto (lx+1, lv-1), is the
  zero function, so A z = 0;
* one-grid sparse grid: the combination technique is the exact inverse, and
  FGMRES converges in one iteration;
* zero input gives zero output.

The prolongation used to build z is written here from the Kuhn refinement
(a fine node 2a + b, b in {0,1}^d, is the midpoint of the coarse edge
a -> a + b), independent of the library and of the oracle.
"""
import sys

import numpy as np
import pytest

from workloads import config_c2, config_c3, config_c5, config_tiny, random_vector
from workloads.configs import lattice_shape

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


def _prolong(c, d, periodic):
    """Kuhn-refinement prolongation of lattice values c (shape m_c^d, trailing
    batch axes allowed after the d lattice axes) to the next level."""
    mc = c.shape[0]
    mf = 2 * mc if periodic else 2 * mc - 1
    idx = np.indices((mf,) * d).reshape(d, -1).T          # fine coordinates
    lo = idx >> 1
    hi = (idx + 1) >> 1
    if periodic:
        lo %= mc
        hi %= mc
    flat = c.reshape((mc ** d,) + c.shape[d:])

    def node(q):
        f = np.zeros(len(q), dtype=np.int64)
        for a in range(d):
            f = f * mc + q[:, a]
        return f
    out = 0.5 * flat[node(lo)] + 0.5 * flat[node(hi)]
    return out.reshape((mf,) * d + c.shape[d:])


def _grid_blocks(ops, y):
    out, off = [], 0
    for _, _, nx, nv in ops.upper:
        n = ops.R * nx * nv
        out.append(y[off:off + n].reshape(ops.R, nx, nv))
        off += n
    return out


@pytest.mark.parametrize("name,fn", [("c2_L7", config_c2), ("c3_L6", config_c3), ("c5_L7", config_c5)])
def test_constants_at_full_size(dev, name, fn):
    from paper_2204_05988_amd import sgdg
    w = fn()
    ops = sgdg.SparseGridOps(w)
    _say(f"constants property {name}: {ops.ndof} DOFs, {len(ops.upper)} grids")
    u = torch.tensor(random_vector(ops.ndof, 41)[0], device=dev)
    y = torch.empty_like(u)
    ops.apply(u, y)
    torch.cuda.synchronize()
    blocks = _grid_blocks(ops, y.cpu().numpy())
    sums = np.array([b.reshape(ops.R, -1).sum(axis=1) for b in blocks])
    scale = max(np.abs(b).sum() for b in blocks)
    err = np.abs(sums - sums[0]).max() / scale
    _say(f"  per-grid sums spread {err:.2e} (relative to sum |y|)")
    assert err <= 1e-12
    ops.close()


@pytest.mark.parametrize("name,fn", [("c2_L7", config_c2), ("c5_L7", config_c5)])
def test_kernel_vectors_at_full_size(dev, name, fn):
    from paper_2204_05988_amd import sgdg
    w = fn()
    ops = sgdg.SparseGridOps(w)
    d, R = w.d, ops.R
    rng = np.random.default_rng(42)
    nup = len(ops.upper)
    worst = 0.0
    for i in [0, nup // 2 - 1, nup - 2]:
        (lx, lv, nx, nv), (lx2, lv2, nx2, nv2) = ops.upper[i], ops.upper[i + 1]
        mx, mvc = lattice_shape(w.x, lx)[0], lattice_shape(w.v, lv - 1)[0]
        c = rng.standard_normal((mx,) * d + (mvc,) * d + (R,))
        # +E^v c on grid i (lx, lv): prolong each x-node's v-lattice
        cv = np.moveaxis(c, list(range(d)), list(range(d + 1, 2 * d + 1)))  # v axes first
        cv = _prolong(cv, d, w.v.periodic)
        cv = np.moveaxis(cv, list(range(d + 1, 2 * d + 1)), list(range(d)))
        # -E^x c on grid i+1 (lx+1, lv-1)
        cx = _prolong(c, d, w.x.periodic)
        blocks = [np.zeros((R, a, b)) for _, _, a, b in ops.upper]
        blocks[i] = np.moveaxis(cv.reshape(nx, nv, R), -1, 0)
        blocks[i + 1] = -np.moveaxis(cx.reshape(nx2, nv2, R), -1, 0)
        z = np.concatenate([b.ravel() for b in blocks])
        zt = torch.tensor(z, device=dev)
        yt = torch.empty_like(zt)
        ops.apply(zt, yt)
        ya = torch.empty_like(zt)
        ops.apply(zt.abs(), ya)
        torch.cuda.synchronize()
        e = yt.abs().max().item() / max(ya.abs().max().item(), 1e-300)
        worst = max(worst, e)
        _say(f"  {name} grids {i},{i + 1}: |A z| / |A |z|| = {e:.2e}")
        assert e <= 1e-12
    ops.close()


def test_one_grid_ct_is_exact(dev):
    from paper_2204_05988_amd import sgdg
    w = config_tiny("d2")
    w.L = w.lmin
    ops = sgdg.SparseGridOps(w)
    assert len(ops.upper) == 1 and len(ops.lower) == 0
    b = torch.tensor(random_vector(ops.ndof, 43)[0], device=dev)
    pc = sgdg.default_precond_opts(inner_rtol=1e-13, inner_maxit=2000)
    x, st = ops.solve_strip(b, torch.zeros_like(b), sgdg.default_solve_opts(rtol=1e-11, pc=pc))
    _say(f"one-grid sparse grid: {st.outer_iters} FGMRES iteration(s), residual {st.rel_residual:.2e}")
    assert st.outer_iters == 1 and st.rel_residual <= 1e-11
    ops.close()


def test_zero_input_and_zero_rhs(dev):
    from paper_2204_05988_amd import sgdg
    w = config_c2(L=4)
    ops = sgdg.SparseGridOps(w)
    u = torch.zeros(2 * ops.ndof, dtype=torch.float64, device=dev)
    y = torch.full_like(u, 7.0)
    ops.apply(u, y, batch=2)
    torch.cuda.synchronize()
    assert torch.count_nonzero(y).item() == 0
    b = torch.zeros(ops.ndof, dtype=torch.float64, device=dev)
    x, st = ops.solve_strip(b, torch.ones_like(b), sgdg.default_solve_opts(rtol=1e-10))
    assert torch.count_nonzero(x).item() == 0 and st.rel_residual == 0.0
    ops.close()
