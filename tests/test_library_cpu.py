"""CPU-side checks of the native library: it loads, exports every declared
entry point, validates arguments before touching a device, and its host
assembly (factor tables, Galerkin restriction, Kronecker term lists) equals
the oracle's operator block by block."""
import os
import re

import numpy as np
import pytest

from paper_2204_05988_amd import sgdg
from workloads import config_c1, config_tiny
from oracle.operator import Problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(sgdg_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = sgdg.lib()
    declared = _declared()
    assert "sgdg_apply_operator" in declared and "sgdg_solve_strip" in declared
    for name in declared:
        assert hasattr(L, name), name


def test_argument_errors_need_no_device():
    import ctypes as C
    L = sgdg.lib()
    dx = sgdg.Domain()
    dx.dim = 2
    dv = sgdg.Domain()
    dv.dim = 3
    g = C.c_void_p()
    assert L.sgdg_build_sparse_grid(C.byref(dx), C.byref(dv), 0, 3, 0, C.byref(g)) == -1
    assert b"dim" in L.sgdg_last_error()
    dv.dim = 2
    for a in range(3):
        dx.hi[a] = dv.hi[a] = 1.0
    assert L.sgdg_build_sparse_grid(C.byref(dx), C.byref(dv), 3, 2, 0, C.byref(g)) == -1
    assert L.sgdg_build_sparse_grid(C.byref(dx), C.byref(dv), 0, 3, 5, C.byref(g)) == -1
    assert L.sgdg_build_sparse_grid(C.byref(dx), C.byref(dv), 0, 3, 1, C.byref(g)) == 0
    n = C.c_int()
    nd = C.c_int64()
    assert L.sgdg_grid_info(g, 0, C.byref(n), C.byref(nd), None, None, None, None, None) == 0
    assert n.value == 4 and nd.value == 2 * (4 * 81 + 9 * 25 + 25 * 9 + 81 * 4)
    assert L.sgdg_grid_info(g, 2, C.byref(n), None, None, None, None, None, None) == -1
    L.sgdg_grid_destroy(g)


@pytest.mark.parametrize("kind", ["d1", "d1p", "d2", "d3"])
def test_host_assembly_equals_oracle(kind):
    w = config_tiny(kind)
    P = Problem(w)
    ops = [(sgdg.OP_FULL, P.terms), (sgdg.OP_MASS, P.mass_terms()), (sgdg.OP_DATA_F, P.data_terms()),
           (sgdg.OP_DATA_G, P.inflow_data_terms())]
    for opk, terms in ops:
        for i in range(len(P.upper)):
            for j in range(len(P.upper)):
                D = sgdg.debug_dense_block(w, opk, i, j)
                O = P.assembled_block(terms, P.upper[i], P.upper[j]).toarray() if terms else 0 * D
                assert np.abs(D - O).max() <= 1e-13 * max(1.0, np.abs(O).max()), (opk, i, j)


def test_host_assembly_c1_cross_blocks():
    """Extreme-aspect blocks of the c1 grid chain (levels 1..6) against the oracle."""
    w = config_c1()
    P = Problem(w)
    n = len(P.upper)
    for i, j in [(0, n - 1), (n - 1, 0), (2, 3), (1, 1)]:
        D = sgdg.debug_dense_block(w, sgdg.OP_FULL, i, j)
        O = P.assembled_block(P.terms, P.upper[i], P.upper[j]).toarray()
        assert np.abs(D - O).max() <= 1e-13 * np.abs(O).max()


def test_fallback_rule_restarts_with_each_fgmres_call():
    """The learned preconditioner's fallback rule measures each FGMRES call
    against its own right-hand side: in mixed precision the second refinement
    step starts at an estimate of O(1) again, which must not be compared with
    the first step's small estimates."""
    # call 0: the network drops the estimate by 10 every 5 iterations (no fallback)
    est0 = [10.0 ** (-(k + 1) / 5) for k in range(12)]
    # call 1 (next refinement step): the same healthy decay from 1 again
    est1 = [10.0 ** (-(k + 1) / 5) for k in range(12)]
    calls = [0] * 12 + [1] * 12
    rel0 = [1.0] * 24
    assert sgdg.debug_fallback(10, 10.0, calls, rel0, est0 + est1) == -1
    # one shared history would compare call 1's O(1) estimates with call 0's 1e-2: a switch at once
    assert sgdg.debug_fallback(10, 10.0, [0] * 24, rel0, est0 + est1) == 12
    # a stagnating network falls back after `iters` learned iterations of its call
    stall = [0.9] * 15
    assert sgdg.debug_fallback(10, 10.0, [0] * 15, [1.0] * 15, stall) == 9
    assert sgdg.debug_fallback(10, 10.0, [0] * 12 + [1] * 15, [1.0] * 27, est0 + stall) == 12 + 9


def test_device_arguments_are_checked_before_any_launch():
    """Every tensor handed to the C ABI is checked for device, contiguity,
    dtype and size first; a wrong buffer must raise, never reach a kernel."""
    torch = pytest.importorskip("torch")
    x = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU"):
        sgdg._dev(x, "u", 10)
    with pytest.raises(TypeError):
        sgdg._dev(np.zeros(10), "u", 10)
    # the checks after the device check, exercised on a stand-in that reports a GPU
    class FakeCuda:
        def __init__(self, t):
            self.t = t
            self.is_cuda = True
            self.dtype = t.dtype

        def is_contiguous(self):
            return self.t.is_contiguous()

        def numel(self):
            return self.t.numel()

        def data_ptr(self):
            return self.t.data_ptr()

    orig = torch.Tensor
    try:
        torch.Tensor = FakeCuda  # isinstance check sees the stand-in as a tensor
        with pytest.raises(ValueError, match="contiguous"):
            sgdg._dev(FakeCuda(torch.zeros(4, 4, dtype=torch.float64).t()), "u", 16)
        with pytest.raises(TypeError, match="dtype"):
            sgdg._dev(FakeCuda(torch.zeros(10, dtype=torch.float32)), "u", 10)
        with pytest.raises(ValueError, match="elements"):
            sgdg._dev(FakeCuda(torch.zeros(9, dtype=torch.float64)), "u", 10)
        assert sgdg._dev(FakeCuda(torch.zeros(10, dtype=torch.float64)), "u", 10) != 0
    finally:
        torch.Tensor = orig
