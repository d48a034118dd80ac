"""Pins of the oracle's block ILU(0) smoother (the smoother of the paper's
experiments, Section 3 and Tables 1-2).

ILU(0) is defined by its pattern: L unit block lower triangular, U block upper
triangular, both on A's pattern of 3x3 blocks, with (L U)_ij = A_ij on every
block of that pattern.  Without fill-in (block tridiagonal A) it is the exact
block LU factorisation; for symmetric A, U = D L^T; for block-diagonal A it is
the block inverse.  The relaxation x <- x + (L U)^{-1} (f - A x) applies
(L U)^{-1} exactly, and on elasticity matrices it contracts (the eigenvalues
of (L U)^{-1} A lie in (0, 2)).  The multicolour variant (block rows in greedy
colour order, the order a GPU triangular solve can take) has a proper
colouring, one dependent step per colour, and converges between block Jacobi
and the natural order.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle
from oracle.setup import ilu0_factors, ilu0_smoother


def _block_tridiagonal(nb, seed):
    rng = np.random.default_rng(seed)
    blocks, cols, ptr = [], [], [0]
    off = [rng.standard_normal((3, 3)) * 0.3 for _ in range(nb - 1)]
    for i in range(nb):
        if i > 0:
            blocks.append(off[i - 1].T)
            cols.append(i - 1)
        g = rng.standard_normal((3, 3))
        blocks.append(g @ g.T + 4.0 * np.eye(3))
        cols.append(i)
        if i + 1 < nb:
            blocks.append(off[i])
            cols.append(i + 1)
        ptr.append(len(cols))
    return sp.csr_matrix(sp.bsr_matrix((np.array(blocks), np.array(cols), np.array(ptr)),
                                       shape=(3 * nb, 3 * nb)))


def _pattern_mask(A):
    B = sp.bsr_matrix(A, blocksize=(3, 3))
    B.data[:] = 1.0
    return sp.csr_matrix(B)


def test_without_fill_ilu0_is_the_exact_block_lu():
    A = _block_tridiagonal(12, seed=1)
    L, U = ilu0_factors(A)
    assert abs(L @ U - A).max() <= 1e-13 * abs(A).max()
    M, _ = ilu0_smoother(A)
    x = np.random.default_rng(2).standard_normal(A.shape[0])
    assert np.linalg.norm(M @ (A @ x) - x) <= 1e-12 * np.linalg.norm(x)


def test_factors_match_a_on_its_pattern_and_have_the_right_shape():
    A = meshgen.cube_c1(5).csr()
    L, U = ilu0_factors(A)
    mask = _pattern_mask(A)
    assert abs((L @ U - A).multiply(mask)).max() <= 1e-13 * abs(A).max()
    Lb, Ub = sp.bsr_matrix(L, blocksize=(3, 3)), sp.bsr_matrix(U, blocksize=(3, 3))
    rows = np.repeat(np.arange(Lb.shape[0] // 3), np.diff(Lb.indptr))
    assert (Lb.indices <= rows).all()
    assert all(np.array_equal(Lb.data[k], np.eye(3)) for k in np.flatnonzero(Lb.indices == rows))
    rows = np.repeat(np.arange(Ub.shape[0] // 3), np.diff(Ub.indptr))
    assert (Ub.indices >= rows).all()
    # no fill: the factors stay inside A's pattern
    assert abs(L.multiply(mask) - L).max() == 0 and abs(U.multiply(mask) - U).max() == 0


def test_symmetric_a_gives_u_equal_d_lt():
    A = meshgen.cube_lognormal(4, seed=3).csr()
    L, U = ilu0_factors(A)
    Ub = sp.bsr_matrix(U, blocksize=(3, 3))
    nb = Ub.shape[0] // 3
    D = np.zeros((nb, 3, 3))
    for i in range(nb):
        for p in range(Ub.indptr[i], Ub.indptr[i + 1]):
            if Ub.indices[p] == i:
                D[i] = Ub.data[p]
    Dm = sp.csr_matrix(sp.bsr_matrix((D, np.arange(nb), np.arange(nb + 1)), shape=A.shape))
    assert abs(U - Dm @ L.T).max() <= 1e-12 * abs(U).max()


def test_block_diagonal_a_gives_the_block_inverse():
    rng = np.random.default_rng(4)
    blocks = np.array([g @ g.T + np.eye(3) for g in rng.standard_normal((7, 3, 3))])
    A = sp.csr_matrix(sp.bsr_matrix((blocks, np.arange(7), np.arange(8)), shape=(21, 21)))
    M, _ = ilu0_smoother(A)
    f = rng.standard_normal(21)
    ref = np.concatenate([np.linalg.solve(blocks[i], f[3 * i:3 * i + 3]) for i in range(7)])
    assert np.allclose(M @ f, ref, rtol=1e-13, atol=1e-13)


def test_apply_inverts_l_u_with_full_diagonal_blocks():
    # U's diagonal blocks are full 3x3 blocks: the apply must not treat U as
    # triangular entry by entry
    A = meshgen.cube_lognormal(5, seed=5).csr()
    L, U = ilu0_factors(A)
    M, _ = ilu0_smoother(A)
    x = np.random.default_rng(6).standard_normal(A.shape[0])
    assert np.linalg.norm(M @ (L @ (U @ x)) - x) <= 1e-12 * np.linalg.norm(x)


def test_relaxation_contracts_and_cuts_the_iterations():
    p = meshgen.cube_c1(6)
    A = p.csr()
    L, U = ilu0_factors(A)
    w = np.linalg.eigvals(np.linalg.solve((L @ U).toarray(), A.toarray()))
    assert abs(w.imag).max() <= 1e-8 and 0 < w.real.min() and w.real.max() < 2
    q = meshgen.cube_c1(10)
    it = {}
    for sm in ("jacobi", "ilu0"):
        h = oracle.build_hierarchy(q.csr(), q.coords, oracle.AmgParams(smoother=sm))
        r = oracle.amg_pcg(h, q.b, tol=1e-8, maxiter=200)
        assert r.converged and r.rel_true_residual <= 1e-8
        it[sm] = r.iters
    assert 2 * it["ilu0"] <= it["jacobi"]       # 9 against 18


def test_greedy_colouring_is_proper_and_optimal_on_bricks():
    from oracle.setup import greedy_block_colouring
    A = meshgen.cube_c1(6).csr()
    colour = greedy_block_colouring(A)
    B = sp.bsr_matrix(A, blocksize=(3, 3))
    rows = np.repeat(np.arange(B.shape[0] // 3), np.diff(B.indptr))
    off = B.indices != rows
    assert (colour[rows[off]] != colour[B.indices[off]]).all()
    # a 2x2x2 cell of nodes is a clique of the 27-point pattern: 8 colours at least
    assert colour.max() + 1 == 8


def test_multicolour_order_gives_one_dependent_step_per_colour():
    from oracle.setup import greedy_block_colouring, ilu0_multicolour_smoother
    A = meshgen.cube_lognormal(5, seed=7).csr()
    colour = greedy_block_colouring(A)
    order = np.argsort(colour, kind="stable")
    perm = (3 * order[:, None] + np.arange(3)[None, :]).ravel()
    Ap = sp.csr_matrix(A[perm][:, perm])
    L, U = ilu0_factors(Ap)
    Lb = sp.bsr_matrix(L, blocksize=(3, 3))
    nb = Lb.shape[0] // 3
    depth = np.zeros(nb, dtype=int)
    for i in range(nb):
        lo = [j for j in Lb.indices[Lb.indptr[i]:Lb.indptr[i + 1]] if j < i]
        depth[i] = 1 + (depth[lo].max() if lo else 0)
    assert depth.max() == colour.max() + 1
    # the smoother applies P^T (L U)^{-1} P exactly
    M, _ = ilu0_multicolour_smoother(A)
    x = np.random.default_rng(8).standard_normal(A.shape[0])
    LUx = np.empty_like(x)
    LUx[perm] = L @ (U @ x[perm])
    assert np.linalg.norm(M @ LUx - x) <= 1e-12 * np.linalg.norm(x)


def test_multicolour_ilu0_converges_between_jacobi_and_natural_order():
    q = meshgen.cube_c1(10)
    it = {}
    for sm in ("jacobi", "ilu0", "ilu0_mc"):
        h = oracle.build_hierarchy(q.csr(), q.coords, oracle.AmgParams(smoother=sm))
        r = oracle.amg_pcg(h, q.b, tol=1e-8, maxiter=200)
        assert r.converged and r.rel_true_residual <= 1e-8
        it[sm] = r.iters
    assert it["ilu0"] < it["ilu0_mc"] < it["jacobi"]       # 9, 16, 18


def _energy_contraction(A, M, iters=60, seed=0):
    """Power estimate of ||I - M A||_A (the A-norm contraction of one sweep):
    below 1 iff every eigenvalue of M A lies in (0, 2)."""
    e = np.random.default_rng(seed).standard_normal(A.shape[0])
    rho = 0.0
    for _ in range(iters):
        y = e - M @ (A @ e)
        ny, ne = np.sqrt(y @ (A @ y)), np.sqrt(e @ (A @ e))
        rho = ny / ne
        e = y / ny
    return rho


@pytest.mark.parametrize("sm", ["ilu0", "ilu0_mc"])
def test_ilu0_contracts_on_every_level_of_a_deep_hierarchy(sm):
    """On aggregate levels the operators are not M-matrices: the sweep must
    still contract in the energy norm there, and CG must converge, with the
    smoother on every level of a four-level hierarchy."""
    q = meshgen.cube_lognormal(12, seed=3)
    h = oracle.build_hierarchy(q.csr(), q.coords, oracle.AmgParams(smoother=sm, coarse_enough=60))
    assert len(h.levels) >= 3
    for lev in h.levels[:-1]:
        rho = _energy_contraction(lev.A, lev.M)
        assert rho < 1.0, (lev.n, rho)
    r = oracle.amg_pcg(h, q.b, tol=1e-8, maxiter=300)
    assert r.converged and r.rel_true_residual <= 1e-8


def test_ilu0_on_the_first_level_only_keeps_block_jacobi_below():
    q = meshgen.cube_lognormal(12, seed=3)
    h = oracle.build_hierarchy(q.csr(), q.coords, oracle.AmgParams(smoother="ilu0_mc", coarse_enough=60,
                                                                   smoother_levels=1))
    J = oracle.build_hierarchy(q.csr(), q.coords, oracle.AmgParams(smoother="jacobi", coarse_enough=60))
    x = np.random.default_rng(1).standard_normal(h.levels[1].n)
    # level 2 carries the block-Jacobi blocks, level 1 does not
    assert np.abs(h.levels[1].M @ x - J.levels[1].M @ x).max() == 0.0
    y = np.random.default_rng(2).standard_normal(h.levels[0].n)
    assert np.abs(h.levels[0].M @ y - J.levels[0].M @ y).max() > 1e-3 * np.abs(J.levels[0].M @ y).max()
