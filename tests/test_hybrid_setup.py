"""The hybrid setup (Section 3: the hierarchy constructed in scalar
arithmetic, every matrix converted to 3x3 blocks afterwards; the paper's
"NS Hybrid" solvers) against the block setup ("NS Block": only the
tentative prolongation in scalar space).  The paper states that both give
identical internal data structures; here every level's A, P and R agree to
rounding, the aggregates are identical, and so are the smoother and fused
operators built from them.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
from paper_2202_09056_amd import HostHierarchy

CASES = {
    "cube10": lambda: (meshgen.cube_c1(10), {}),
    "lognormal16_3lvl": lambda: (meshgen.cube_lognormal(16, seed=0), {"coarse_enough": 300}),
    "tets12": lambda: (meshgen.tet_cube(12), {"coarse_enough": 300}),
    "beam32x4x4": lambda: (meshgen.beam(32, 4, 4), {"coarse_enough": 200}),
    "no_nullspace": lambda: (meshgen.cube_c1(8), {"use_nullspace": 0, "coarse_enough": 300}),
    "spai0": lambda: (meshgen.cube_lognormal(12, seed=1), {"smoother": "spai0"}),
}


def _rel(a, b):
    d = abs(a - b).max() if (a - b).nnz else 0.0
    return d / max(abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", list(CASES))
def test_scalar_then_convert_equals_block_setup(name):
    p, kw = CASES[name]()
    Hb = HostHierarchy(p.row_ptr, p.col, p.val, p.coords, **kw)
    Hs = HostHierarchy(p.row_ptr, p.col, p.val, p.coords, setup_path="scalar", **kw)
    sb, ss = Hb.stats(), Hs.stats()
    assert sb.levels == ss.levels >= 2
    for l in range(sb.levels):
        assert sb.nb[l] == ss.nb[l]
        assert _rel(Hs.scipy(l, "A"), Hb.scipy(l, "A")) <= 1e-13
        if l + 1 < sb.levels:
            assert np.array_equal(Hs.aggregates(l), Hb.aggregates(l))
            for op in ("P", "R", "G"):
                assert _rel(Hs.scipy(l, op), Hb.scipy(l, op)) <= 1e-13, (l, op)
            Mb, Ms = Hb.smoother_blocks(l), Hs.smoother_blocks(l)
            assert np.abs(Ms - Mb).max() <= 1e-12 * np.abs(Mb).max()
    # the setup phases are timed; only the hybrid path converts
    assert all(v >= 0 for v in ss.setup_phase_ms) and all(v >= 0 for v in sb.setup_phase_ms)
    assert ss.setup_phase_ms[10] > 0 and sb.setup_phase_ms[10] == 0
    assert abs(sum(ss.setup_phase_ms) - ss.setup_ms) <= 0.05 * ss.setup_ms + 1.0


def test_scalar_kernels_round_trip():
    """unblock/reblock through the library's export: the scalar hierarchy's
    operators are the block ones with the same values (checked above); here the
    exact-zero handling: a block with zeros keeps its pattern in block form."""
    p = meshgen.cube_c1(5)
    H = HostHierarchy(p.row_ptr, p.col, p.val, p.coords, setup_path="scalar", coarse_enough=100)
    A = H.scipy(0, "A")
    ref = sp.bsr_matrix((p.val.reshape(-1, 3, 3), p.col, p.row_ptr), shape=A.shape).tocsr()
    assert abs(A - ref).max() == 0.0
