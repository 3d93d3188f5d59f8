"""The split passes stage W, Pt and Qt only where they are read (face terms
near their face).  Whatever the shared work buffers hold elsewhere must never
reach a result: the buffers are first filled with NaN by applies of a NaN
vector in the configurations that write them everywhere (box-tiled kernel:
dense partner arrays; one vector per thread: W everywhere), then a finite
vector is applied in every split configuration and compared with the oracle."""
import sys

import numpy as np
import pytest

from workloads import config_c2, config_c5, random_vector
from oracle.operator import Problem

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


@pytest.mark.parametrize("name", ["c2_L5", "c5_L4"])
def test_stale_buffers_never_reach_results(dev, name):
    from paper_2204_05988_amd import sgdg
    w = config_c2(L=5) if name == "c2_L5" else config_c5(L=4)
    P = Problem(w)
    ops = sgdg.SparseGridOps(w)
    B = 2
    u = random_vector(P.ndof, 23, batch=B)
    ref = np.stack([P.apply(u[b]) for b in range(B)])
    for dt, tol in (("f64", 1e-10), ("f32", 1e-4)):
        tdt = torch.float64 if dt == "f64" else torch.float32
        bad = torch.full((B, P.ndof), float("nan"), dtype=tdt, device=dev)
        y = torch.empty_like(bad)
        for cfg in (("fused", 0, 8, 0), ("split", 1, 8, 0)):
            ops.set_launch(*cfg)
            ops.apply(bad, y, batch=B)
        torch.cuda.synchronize()
        assert torch.isnan(y).all()
        ut = torch.tensor(u, device=dev, dtype=tdt)
        for cfg in (("split", 2, 8, 0), ("split_tiled", 2, 8, 0), ("split", 2, 8, 1), ("split_tiled", 1, 8, 0)):
            _say(f"{name} {dt} {cfg}")
            ops.set_launch(*cfg)
            ops.apply(ut, y, batch=B)
            torch.cuda.synchronize()
            yy = y.double().cpu().numpy()
            assert np.isfinite(yy).all(), cfg
            err = np.abs(yy - ref).max() / np.abs(ref).max()
            assert err <= tol, (cfg, err)
            # poison again between configurations
            for pcfg in (("fused", 0, 8, 0), ("split", 1, 8, 0)):
                ops.set_launch(*pcfg)
                ops.apply(bad, y, batch=B)
    ops.close()
