"""Host setup of the block ILU(0) smoother (CPU, no GPU): the library's
multicolour order and incomplete factors against the oracle's, built
independently from the same matrices (Section 3: ILU(0) with 3x3 block
values, the smoother of the paper's experiments)."""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle
from oracle.setup import greedy_block_colouring, ilu0_factors
from paper_2202_09056_amd import HostHierarchy, AmgError

CASES = {
    "cube10": lambda: (meshgen.cube_c1(10), {}),
    "lognormal14": lambda: (meshgen.cube_lognormal(14, seed=0), {}),
    "tets12": lambda: (meshgen.tet_cube(12), {"coarse_enough": 300}),
    "lognormal12_all_levels": lambda: (meshgen.cube_lognormal(12, seed=2), {"coarse_enough": 100,
                                                                           "smoother_levels": 0}),
}


def _permuted_factors(A, colour):
    """Oracle factors in the colour order, mapped back to the level's numbering."""
    order = np.argsort(colour, kind="stable")
    perm = (3 * order[:, None] + np.arange(3)[None, :]).ravel()
    Ap = sp.csr_matrix(A[perm][:, perm])
    Ap.sort_indices()
    Lp, Up = ilu0_factors(Ap)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(A.shape[0])
    back = lambda M: sp.csr_matrix(M[inv][:, inv])
    return back(Lp - sp.identity(A.shape[0], format="csr")), back(Up)


@pytest.mark.parametrize("name", list(CASES))
def test_ilu0_colours_and_factors_match_oracle(name):
    p, kw = CASES[name]()
    H = HostHierarchy(p.row_ptr, p.col, p.val, p.coords, smoother="ilu0", **kw)
    nlev = H.levels
    assert nlev >= 2
    ilu_levels = kw.get("smoother_levels", 1) or (nlev - 1)
    for l in range(nlev - 1):
        colours = H.ilu_colours(l)
        if l >= ilu_levels:
            assert colours is None
            continue
        A = H.scipy(l, "A")
        ref = greedy_block_colouring(A)
        assert np.array_equal(colours, ref)
        Lo, Uo = _permuted_factors(A, ref)
        L = H.scipy(l, "ILU_L")
        U = H.scipy(l, "ILU_U")
        scale = abs(Uo).max()
        assert abs(L - Lo).max() <= 1e-12 * max(abs(Lo).max(), 1.0)
        assert abs(U - Uo).max() <= 1e-12 * scale
        # L couples a row only to lower colours, U (off its diagonal) only to higher ones
        for M, lower in ((L, True), (U, False)):
            coo = M.tocoo()
            I, J = coo.row // 3, coo.col // 3
            off = I != J
            assert np.all((colours[J[off]] < colours[I[off]]) == lower)
        # L U reproduces A on A's block pattern (the defining property of ILU(0))
        LU = (L + sp.identity(A.shape[0])) @ U
        Ab = sp.bsr_matrix(A, blocksize=(3, 3))
        mask = sp.bsr_matrix((np.ones_like(Ab.data), Ab.indices, Ab.indptr), shape=A.shape).tocsr()
        diff = (LU - A).multiply(mask)
        assert abs(diff).max() <= 1e-12 * abs(A).max()


def test_ilu0_levels_below_use_block_jacobi():
    p = meshgen.cube_lognormal(12, seed=1)
    H = HostHierarchy(p.row_ptr, p.col, p.val, p.coords, smoother="ilu0", coarse_enough=100)
    st = H.stats()
    assert st.levels >= 3
    assert H.ilu_colours(0) is not None and H.ilu_colours(1) is None
    # level 2 keeps the fused sweeps of block Jacobi, level 1 has none
    assert H.bsr(0, "G")[1].size == 0 and H.bsr(1, "G")[1].size > 0


def test_ilu0_rejects_negative_level_count():
    p = meshgen.cube_c1(4)
    with pytest.raises(AmgError):
        HostHierarchy(p.row_ptr, p.col, p.val, p.coords, smoother="ilu0", smoother_levels=-1)
