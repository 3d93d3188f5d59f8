"""Where the X-factors can contribute (sgdg_op_support), checked against the
lattice geometry: on the c2 problem the four x-face masses (Sect. 4.2's
boundary terms of the inflow boundary) are nonzero on their own face only;
with x periodic (c5) only the kinked-field weights of the v-face terms leave
nodes out."""
import pytest

from workloads import config_c2, config_c5

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sg():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_05988_amd import sgdg
    sgdg.lib()
    return sgdg


def test_face_masses_live_on_their_face(sg):
    ops = sg.SparseGridOps(config_c2(L=5))
    nxg = ops.op_info()["nxg"]
    for lx in range(0, 6):
        m = 2 ** lx + 1  # nodes per axis of the 2D x-lattice
        c = ops.op_support(lx)
        assert c["nodes"] == m * m
        # 4 face groups: rows on the m nodes of their face; the x-stencil of
        # those rows reads the face and the next line in (both for m >= 2)
        faces = 4
        assert c["row_groups"] == (nxg - faces) * m * m + faces * m, (lx, c)
        assert c["read_groups"] == (nxg - faces) * m * m + faces * min(2 * m, m * m), (lx, c)
        # Qt^m (restriction of the finer level's X_m u) can be nonzero only on
        # the coarse face; the coarsest level sees all of its nodes
        assert c["qt_groups"] <= nxg * m * m
        if lx < 5:
            assert c["qt_groups"] == (nxg - faces) * m * m + faces * m, (lx, c)
        assert c["read_terms"] >= c["read_groups"] and c["qt_terms"] >= c["qt_groups"]
    ops.close()


def test_periodic_x_has_no_faces(sg):
    # x periodic: no x-faces.  The v-face terms carry x-factors weighted by a
    # kinked field, max(-E.n, 0) for the four v-faces, which vanish where E.n
    # is positive on a node's whole support; every other factor covers every node.
    ops = sg.SparseGridOps(config_c5(L=4))
    info = ops.op_info()
    nxg = info["nxg"]
    partial_levels = 0
    for lx in range(0, 5):
        c = ops.op_support(lx)
        n = c["nodes"]
        assert n == (2 ** lx) ** 2
        assert (nxg - 4) * n <= c["row_groups"] <= c["read_groups"] <= nxg * n, (lx, c)
        assert c["qt_groups"] <= nxg * n
        partial_levels += c["row_groups"] < nxg * n
    assert partial_levels > 0  # the random field changes sign within the finer lattices
    ops.close()
