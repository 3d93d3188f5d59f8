"""The allocation-free operator application (sgdg_apply_operator_noalloc)
against the ordinary entry point, through the C ABI.

It runs the same kernels with its work arrays carved from one fixed device
array, so its results must equal sgdg_apply_operator's bit for bit (and the
oracle to 1e-10 in FP64).  Two calls in a row, the second with a smaller
input, check that the shared array's leftover contents never leak into a
result; the call must allocate nothing (the device's free memory does not
change across it) and must refuse work beyond its array.
"""
import sys

import numpy as np
import pytest

from workloads import config_c2, config_tiny, random_vector
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


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("launch", [("split", 2, 8, 0), ("split_tiled", 2, 8, 1), ("fused", 0, 8, 0)],
                         ids=["split", "tiled", "fused"])
def test_noalloc_apply_equals_apply(dev, launch):
    from paper_2204_05988_amd import sgdg
    w = config_c2(L=5)
    P = Problem(w)
    ops = sgdg.SparseGridOps(w)
    ops.set_launch(*launch)
    for dt in (torch.float64, torch.float32):
        for call, B in enumerate((4, 2)):      # second call: smaller input
            u = torch.tensor(random_vector(P.ndof, 60 + call, batch=B), device=dev, dtype=dt)
            y_ref = torch.empty_like(u)
            _say(f"no-alloc apply {launch} {dt} call {call} batch {B}")
            ops.apply(u, y_ref, batch=B)           # builds the tables (first call) and is the reference
            torch.cuda.synchronize()
            y = torch.full_like(u, float("nan"))
            ops.apply_noalloc(u, y, batch=B)
            torch.cuda.synchronize()
            assert torch.equal(y, y_ref)
            if dt == torch.float64:
                for b in (0, B - 1):
                    assert _rel(y[b].cpu().numpy(), P.apply(u[b].cpu().numpy())) <= 1e-10
    ops.close()


def test_noalloc_other_kinds_and_errors(dev):
    from paper_2204_05988_amd import sgdg
    w = config_tiny("d2")
    ops = sgdg.SparseGridOps(w)
    u = torch.tensor(random_vector(ops.ndof, 5)[0], device=dev)
    y = torch.empty_like(u)
    # tables of a kind are built by its first ordinary application
    with pytest.raises(sgdg.SgdgError) as ei:
        ops.apply_noalloc(u, y, sgdg.OP_DATA_F)
    assert ei.value.code == -7
    for kind in (sgdg.OP_FULL, sgdg.OP_BLOCKDIAG, sgdg.OP_DATA_F):
        yr = torch.empty_like(u)
        ops.apply(u, yr, kind)
        ops.apply_noalloc(u, y, kind)
        torch.cuda.synchronize()
        assert torch.equal(y, yr), kind
    # beyond the fixed array: a clear error, nothing launched
    wbig = config_c2(L=7)
    big = sgdg.SparseGridOps(wbig)
    ub = torch.zeros(big.ndof, dtype=torch.float64, device=dev)
    yb = torch.empty_like(ub)
    big.apply(ub, yb)
    B = 64
    ubb = torch.zeros(B * big.ndof, dtype=torch.float32, device=dev)
    ybb = torch.empty_like(ubb)
    big.apply(ubb[:big.ndof], ybb[:big.ndof])    # FP32 tables
    with pytest.raises(sgdg.SgdgError) as ei:
        big.apply_noalloc(ubb, ybb, batch=B)
    assert ei.value.code == -1 and "bytes of scratch" in str(ei.value)
    # one FP64 vector of the level-7 problem fits, and a call allocates nothing:
    # the device's free memory is the same before and after it
    big.apply_noalloc(ub, yb)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    big.apply_noalloc(ub, yb)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert torch.equal(yb, torch.zeros_like(yb))
    big.close()
    ops.close()
