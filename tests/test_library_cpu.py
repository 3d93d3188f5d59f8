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
