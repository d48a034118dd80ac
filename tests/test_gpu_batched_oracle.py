"""The batched forms applied once, column by column and problem by problem,
against the oracle's V-cycle (Algorithm 2), entry by entry.

* Multi-column V-cycle (block SpMM: every operator read once for all
  columns): each of k = 1, 4, 7, 12, 32 columns equals the oracle's V-cycle
  of that column (FP64; FP32 within its rounding, k = 5 and 8).  In FP64 the
  even k take the 16-byte column-vector kernels (two columns per lane), the
  odd k the one-column-per-lane kernels.
* Batched V-cycle (every problem's level operators concatenated, one launch
  per step): each problem of a batch of mixed sizes and depths equals the
  oracle's V-cycle of its own hierarchy.
* The coarsest solve for k columns (FP64 MFMA GEMM with the explicit inverse)
  equals the oracle's Cholesky solve of every column, on a hierarchy that is
  only the coarsest level.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import meshgen
import oracle

from parity import assert_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_09056_amd import Solver, BatchSolver  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("k", [1, 4, 7, 12, 32])
def test_multi_column_vcycle_matches_oracle_per_column(k):
    p = meshgen.cube_lognormal(16, seed=5)
    h = oracle.build_hierarchy(p.csr(), p.coords, oracle.AmgParams(coarse_enough=300))
    assert len(h.levels) == 3
    s = Solver(p.row_ptr, p.col, p.val, p.coords, coarse_enough=300)
    rng = np.random.default_rng(30 + k)
    R = rng.standard_normal((p.n, k))
    Z = s.vcycle_multi(_dev(R)).cpu().numpy()
    s.close()
    for j in range(k):
        assert_close(Z[:, j], oracle.vcycle(h, R[:, j]), 1e-10, 1e-12, f"column {j} of {k}")


@pytest.mark.parametrize("k", [5, 8])
def test_multi_column_vcycle_fp32_within_rounding(k):
    p = meshgen.cube_lognormal(14, seed=6)
    h = oracle.build_hierarchy(p.csr(), p.coords)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, precision="fp32")
    R = np.random.default_rng(40).standard_normal((p.n, k))
    Z = s.vcycle_multi(_dev(R)).cpu().numpy()
    s.close()
    for j in range(k):
        ref = oracle.vcycle(h, R[:, j])
        assert np.linalg.norm(Z[:, j] - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("k", [1, 7, 32])
def test_coarsest_gemm_matches_cholesky_per_column(k):
    """Single-level hierarchy: the V-cycle is the dense coarsest solve, here
    the FP64 MFMA GEMM with the explicit inverse, for k columns at once."""
    p = meshgen.cube_lognormal(8, seed=7)   # 2187 unknowns <= 3000: one level
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    assert s.stats().levels == 1
    R = np.random.default_rng(50 + k).standard_normal((p.n, k))
    Z = s.vcycle_multi(_dev(R)).cpu().numpy()
    s.close()
    c = sla.cho_factor(A.toarray(), lower=True)
    for j in range(k):
        assert_close(Z[:, j], sla.cho_solve(c, R[:, j]), 1e-10, 1e-12, f"coarsest column {j}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_vcycle_matches_oracle_per_problem(prec):
    # single-level, two-level and three-level problems of different sizes,
    # bricks and tetrahedra, in one batch
    probs = [meshgen.cube_c1(4), meshgen.cube_lognormal(9, seed=4), meshgen.cube_c1(12),
             meshgen.tet_cube(9), meshgen.cube_lognormal(14, seed=8)]
    prm = dict(coarse_enough=400)
    hs = [oracle.build_hierarchy(q.csr(), q.coords, oracle.AmgParams(**prm)) for q in probs]
    assert sorted({len(h.levels) for h in hs}) == [1, 2, 3]
    bat = BatchSolver([(q.row_ptr, q.col, q.val, q.coords) for q in probs], precision=prec, **prm)
    rng = np.random.default_rng(60)
    rs = [rng.standard_normal(q.n) for q in probs]
    zs = bat.vcycle([_dev(r) for r in rs])
    bat.close()
    for i, (h, r, z) in enumerate(zip(hs, rs, zs)):
        ref = oracle.vcycle(h, r)
        got = z.cpu().numpy()
        if prec == "fp64":
            assert_close(got, ref, 1e-10, 1e-12, f"problem {i} ({len(h.levels)} levels)")
        else:
            assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref), i


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_column_forms_on_long_rows(prec):
    """A level-2 operator (about 60 blocks per row) taken as the system
    matrix, so that the level-1 products of the multi-column path, the
    reducing ones included (q = A p with its column dots, the initial
    residual norms), take the workgroup-per-row kernel: the multi-column
    V-cycle equals the single-vector V-cycle of each column (FP64 to 1e-10
    entry-wise), and every column of a multi-right-hand-side solve meets the
    FP64 true residual and its own single solve's iteration count within one."""
    from paper_2202_09056_amd import HostHierarchy
    import scipy.sparse as sp
    q = meshgen.cube_lognormal(16, seed=0)
    H = HostHierarchy(q.row_ptr, q.col, q.val, q.coords, coarse_enough=300)
    rp, col, val, (rows, cols) = H.bsr(1, "A")
    H.close()
    assert col.size / rows > 32                          # long rows on the finest level
    A = sp.bsr_matrix((val, col, rp), shape=(3 * rows, 3 * rows)).tocsr()
    coords = np.zeros((rows, 3))
    s = Solver(rp, col, val, coords, use_nullspace=0, coarse_enough=300, precision=prec)
    k = 4
    rng = np.random.default_rng(70)
    R = rng.standard_normal((3 * rows, k))
    Z = s.vcycle_multi(_dev(R)).cpu().numpy()
    for j in range(k):
        zj = s.vcycle(_dev(R[:, j])).cpu().numpy()
        if prec == "fp64":
            assert_close(Z[:, j], zj, 1e-10, 1e-12, f"long rows, column {j}")
        else:
            assert np.linalg.norm(Z[:, j] - zj) <= 1e-5 * np.linalg.norm(zj)
    X, infos, status = s.solve_multi(_dev(R), tol=1e-8)
    assert status == 0
    Xh = X.cpu().numpy()
    for j in range(k):
        assert infos[j].converged == 1
        assert oracle.true_residual_norm(A, R[:, j], Xh[:, j]) <= 1e-8
        _, i1, _ = s.solve(_dev(R[:, j]), tol=1e-8)
        assert abs(i1.iters - infos[j].iters) <= 1, (j, i1.iters, infos[j].iters)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_coarsest_solves_of_the_largest_size(prec):
    """Problems small enough to be solved directly (up to 3000 unknowns, the
    default coarse_enough): their batched V-cycle is the coarsest solve alone,
    y = S f with the dense inverse S (2187, 3000 and 1029 unknowns, rows
    longer than a wavefront's 64 lanes many times over), against a Cholesky
    solve of the same matrix."""
    probs = [meshgen.cube_c1(8), meshgen.cube_lognormal(9, seed=5), meshgen.cube_c1(6)]
    assert [q.n for q in probs] == [2187, 3000, 1029]
    bat = BatchSolver([(q.row_ptr, q.col, q.val, q.coords) for q in probs], precision=prec)
    rng = np.random.default_rng(61)
    rs = [rng.standard_normal(q.n) for q in probs]
    zs = bat.vcycle([_dev(r) for r in rs])
    bat.close()
    for i, (q, r, z) in enumerate(zip(probs, rs, zs)):
        ref = sla.cho_solve(sla.cho_factor(q.csr().toarray()), r)
        got = z.cpu().numpy()
        if prec == "fp64":
            assert_close(got, ref, 1e-10, 1e-12, f"problem {i} ({q.n} unknowns)")
        else:
            assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref), i
