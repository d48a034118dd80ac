"""GPU checks of the batched forms.

Batch of independent problems (one launch per V-cycle step for the whole
batch, per-problem CG scalars): every problem must match its own single
solve (iterations within one, same FP64 residual target, direct solution),
for sizes from single-level (dense) to three-level hierarchies.

Multi-right-hand-side solve (block SpMM, per-column CG): every column must
reach the FP64 true residual target (recomputed by scipy), agree with the
direct solution, and take the same number of iterations (within one) as the
single-vector solve of that column; a zero column stays zero; columns that
converge early are frozen.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import meshgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_09056_amd import Solver, BatchSolver  # noqa: E402
from paper_2202_09056_amd import _capi  # noqa: E402


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("k", [1, 7, 32])
def test_multi_rhs_matches_single_solves(prec, k):
    p = meshgen.cube_lognormal(12, seed=3)
    A = p.csr()
    rng = np.random.default_rng(10 + k)
    B = rng.standard_normal((p.n, k))
    B[np.repeat(p.fixed, 3)] = 0.0
    B[:, 0] = p.b                      # a smooth load next to random ones
    if k > 2:
        B[:, 2] = 0.0                  # a zero right-hand side
    s = Solver(p.row_ptr, p.col, p.val, p.coords, precision=prec)
    Bd = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    X, infos, status = s.solve_multi(Bd, tol=1e-8)
    assert status == _capi.AMG_OK
    Xh = X.cpu().numpy()
    lu = spla.splu(A.tocsc())
    for j in range(k):
        if not B[:, j].any():
            assert not Xh[:, j].any() and infos[j].iters == 0
            continue
        assert infos[j].converged == 1
        assert oracle.true_residual_norm(A, B[:, j], Xh[:, j]) <= 1e-8
        assert _rel(Xh[:, j], lu.solve(B[:, j])) <= 1e-6
        x1, i1, st1 = s.solve(torch.from_numpy(np.ascontiguousarray(B[:, j])).cuda(), tol=1e-8)
        assert abs(i1.iters - infos[j].iters) <= 1, (j, i1.iters, infos[j].iters)
        assert _rel(Xh[:, j], x1.cpu().numpy()) <= 1e-6
    s.close()


def test_multi_rhs_warm_start_and_repeat():
    p = meshgen.cube_c1(10)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, precision="fp32")
    B = torch.from_numpy(np.ascontiguousarray(np.stack([p.b, 2 * p.b], axis=1))).cuda()
    X, infos, status = s.solve_multi(B)
    X2, infos2, status2 = s.solve_multi(B, X.clone())
    assert status2 == 0 and all(i.iters == 0 for i in infos2)
    X3, infos3, _ = s.solve_multi(B)
    assert torch.equal(X, X3)  # deterministic
    np.testing.assert_allclose(X[:, 1].cpu().numpy(), 2 * X[:, 0].cpu().numpy(), rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_problem_batch_matches_single_solves(prec):
    probs = [meshgen.cube_c1(3), meshgen.cube_lognormal(12, seed=1), meshgen.cube_c1(10),
             meshgen.cube_c1(4), meshgen.cube_lognormal(20, seed=2), meshgen.cube_c1(8)]
    bs = [torch.from_numpy(np.ascontiguousarray(p.b)).cuda() for p in probs]
    B = BatchSolver([(p.row_ptr, p.col, p.val, p.coords) for p in probs], precision=prec)
    xs, infos, status = B.solve(bs, tol=1e-8)
    assert status == _capi.AMG_OK
    for p, x, inf in zip(probs, xs, infos):
        A = p.csr()
        xh = x.cpu().numpy()
        assert inf.converged == 1
        assert oracle.true_residual_norm(A, p.b, xh) <= 1e-8
        assert _rel(xh, spla.splu(A.tocsc()).solve(p.b)) <= 1e-6
        s = Solver(p.row_ptr, p.col, p.val, p.coords, precision=prec)
        x1, i1, _ = s.solve(torch.from_numpy(np.ascontiguousarray(p.b)).cuda(), tol=1e-8)
        assert abs(i1.iters - inf.iters) <= 1, (p.name, i1.iters, inf.iters)
        s.close()
    # a second solve reuses the captured graph and gives the same answer
    xs2, infos2, status2 = B.solve(bs, tol=1e-8)
    assert status2 == 0 and all(torch.equal(a, b) for a, b in zip(xs, xs2))
    B.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_rhs_beyond_one_grid_sweep(prec):
    """A level with more block rows than one sweep of the capped multi-column
    grid (2048 workgroups x 8 rows): every row must still be visited by every
    kernel of the multi-column V-cycle (iterations equal the single solves)."""
    p = meshgen.cube_c1(26)                  # 19,683 block rows
    assert p.n // 3 > 2048 * 8
    s = Solver(p.row_ptr, p.col, p.val, p.coords, precision=prec)
    rng = np.random.default_rng(30)
    B = rng.standard_normal((p.n, 4)) * np.repeat(~p.fixed, 3)[:, None]
    X, infos, status = s.solve_multi(torch.from_numpy(np.ascontiguousarray(B)).cuda(), tol=1e-8)
    assert status == _capi.AMG_OK
    A = p.csr()
    Xh = X.cpu().numpy()
    for j in range(4):
        assert oracle.true_residual_norm(A, B[:, j], Xh[:, j]) <= 1e-8
        _, i1, _ = s.solve(torch.from_numpy(np.ascontiguousarray(B[:, j])).cuda(), tol=1e-8)
        assert abs(i1.iters - infos[j].iters) <= 1, (j, i1.iters, infos[j].iters)
    s.close()


@pytest.mark.parametrize("smoother", ["learned", "spai0", "jacobi"])
def test_multi_rhs_with_fused_and_plain_levels(smoother):
    """Three levels whose sweeps are fused (G, AM) on some levels and plain on
    others: the learned context keeps level 1 plain (its blocks change after
    setup), SPAI-0 fuses every level with its two block sets (M, M^T), block
    Jacobi fuses all.  Every column matches its single solve within one
    iteration."""
    p = meshgen.cube_lognormal(22, seed=0)
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother=smoother)
    st = s.stats()
    assert st.levels == 3
    rng = np.random.default_rng(8)
    B = rng.standard_normal((p.n, 4))
    B[np.repeat(p.fixed, 3)] = 0.0
    X, infos, status = s.solve_multi(torch.from_numpy(np.ascontiguousarray(B)).cuda(), tol=1e-8)
    assert status == _capi.AMG_OK
    Xh = X.cpu().numpy()
    for j in range(B.shape[1]):
        assert infos[j].converged == 1
        assert oracle.true_residual_norm(A, B[:, j], Xh[:, j]) <= 1e-8
        _, i1, _ = s.solve(torch.from_numpy(np.ascontiguousarray(B[:, j])).cuda(), tol=1e-8)
        assert abs(i1.iters - infos[j].iters) <= 1, (smoother, j, i1.iters, infos[j].iters)
    s.close()
