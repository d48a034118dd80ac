"""GPU parity of the block SPAI-0 smoother (pre-sweep M, post-sweep M^T),
run through the two-block fused post-sweep z = G e + M f + M^T t.

The library and the oracle build their own SPAI-0 hierarchies from the same
inputs.  FP64: the V-cycle agrees with the oracle's to 1e-11 (the same bound
as block Jacobi: identical operators up to summation order) and CG takes the
oracle's iteration count within one.  The reduced-precision, multi-RHS and
batch forms reach the FP64 true residual 1e-8 and match their single FP64
solves within one iteration (multi-RHS, batch) or converge (FP32 V-cycle,
whose count moves with rounding).
"""
import numpy as np
import pytest

import meshgen
import oracle

from parity import assert_close, assert_close_scaled

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_09056_amd import Solver, BatchSolver  # noqa: E402
from paper_2202_09056_amd import _capi  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = {
    "cube10": lambda: meshgen.cube_c1(10),
    "lognormal14": lambda: meshgen.cube_lognormal(14, seed=0),
    "inclusions16": lambda: meshgen.cube_inclusions(16, n_incl=8, radius_elems=2.5),
    "lognormal22": lambda: meshgen.cube_lognormal(22, seed=0),  # three levels: fused sweeps below the first
}


@pytest.mark.parametrize("name", list(CASES))
def test_spai0_vcycle_and_solve_match_oracle(name):
    p = CASES[name]()
    print(f"[spai0] {name} n={p.n}", flush=True)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords, oracle.AmgParams(smoother="spai0"))
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="spai0")
    assert s.stats().levels == len(h.levels)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(p.n)
    assert_close(s.vcycle(_dev(r)).cpu().numpy(), oracle.vcycle(h, r), 1e-10, 1e-11, "V-cycle")
    ref = oracle.amg_pcg(h, p.b, tol=1e-8, maxiter=3000)
    x, info, status = s.solve(_dev(p.b), tol=1e-8)
    s.close()
    print(f"[spai0] {name}: gpu iters={info.iters} oracle iters={ref.iters}", flush=True)
    assert status == _capi.AMG_OK and info.converged == 1
    assert abs(info.iters - ref.iters) <= 1
    assert oracle.true_residual_norm(A, p.b, x.cpu().numpy()) <= 1e-8


def test_spai0_post_sweep_uses_the_transpose():
    # with M^T on the post-sweep the V-cycle is a symmetric operator: <V a, b> = <a, V b>
    p = meshgen.cube_lognormal(10, seed=2)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="spai0", coarse_enough=300)
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(p.n), rng.standard_normal(p.n)
    va = s.vcycle(_dev(a)).cpu().numpy()
    vb = s.vcycle(_dev(b)).cpu().numpy()
    s.close()
    assert abs(va @ b - a @ vb) <= 1e-12 * np.linalg.norm(va) * np.linalg.norm(b)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_spai0_reduced_precision_converges(prec):
    p = meshgen.cube_lognormal(16, seed=1)
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="spai0", precision=prec)
    x, info, status = s.solve(_dev(p.b), tol=1e-8)
    s.close()
    assert status == _capi.AMG_OK and info.converged == 1
    assert oracle.true_residual_norm(A, p.b, x.cpu().numpy()) <= 1e-8


def test_spai0_multi_rhs_and_batch_match_single_solves():
    p = meshgen.cube_lognormal(12, seed=3)
    A = p.csr()
    rng = np.random.default_rng(6)
    B = rng.standard_normal((p.n, 5))
    B[np.repeat(p.fixed, 3)] = 0.0
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="spai0")
    X, infos, status = s.solve_multi(_dev(B), tol=1e-8)
    assert status == _capi.AMG_OK
    Xh = X.cpu().numpy()
    for j in range(B.shape[1]):
        assert oracle.true_residual_norm(A, B[:, j], Xh[:, j]) <= 1e-8
        _, i1, _ = s.solve(_dev(B[:, j]), tol=1e-8)
        assert abs(i1.iters - infos[j].iters) <= 1, (j, i1.iters, infos[j].iters)
    s.close()
    probs = [meshgen.cube_c1(6), meshgen.cube_lognormal(9, seed=4), meshgen.cube_c1(12)]
    bs = [_dev(q.b) for q in probs]
    bat = BatchSolver([(q.row_ptr, q.col, q.val, q.coords) for q in probs], smoother="spai0")
    xs, binfos, status = bat.solve(bs, tol=1e-8)
    bat.close()
    assert status == _capi.AMG_OK
    for q, x, inf in zip(probs, xs, binfos):
        assert oracle.true_residual_norm(q.csr(), q.b, x.cpu().numpy()) <= 1e-8
        s1 = Solver(q.row_ptr, q.col, q.val, q.coords, smoother="spai0")
        _, i1, _ = s1.solve(_dev(q.b), tol=1e-8)
        s1.close()
        assert abs(i1.iters - inf.iters) <= 1, (i1.iters, inf.iters)


def test_spai0_fused_kernels_match_oracle_operators():
    """The two-block fused post-sweep z = G e + M f + M^T t and the fused
    residual t = f - A M f on every level, against the oracle's SPAI-0
    operators (M and its transpose on the post-sweep)."""
    p = meshgen.cube_lognormal(22, seed=0)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords, oracle.AmgParams(smoother="spai0"))
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="spai0")
    rng = np.random.default_rng(12)
    for l in range(len(h.levels) - 1):
        lev, nxt = h.levels[l], h.levels[l + 1]
        f, t, e = rng.standard_normal(lev.n), rng.standard_normal(lev.n), rng.standard_normal(nxt.n)
        out = _dev(t)
        s.debug_apply(l, 12, _dev(e), out, in2=_dev(f))
        pe = lev.P @ e
        ref = pe - lev.Mt @ (lev.A @ pe) + lev.M @ f + lev.Mt @ t
        ape = abs(lev.P) @ np.abs(e)
        scale = ape + abs(lev.Mt) @ (abs(lev.A) @ ape) + abs(lev.M) @ np.abs(f) + abs(lev.Mt) @ np.abs(t)
        assert_close_scaled(out.cpu().numpy(), ref, scale, 1e-12, f"post level {l}")
        if l > 0:
            s.debug_apply(l, 11, _dev(f), out)
            scale = np.abs(f) + abs(lev.A) @ (abs(lev.M) @ np.abs(f))
            assert_close_scaled(out.cpu().numpy(), f - lev.A @ (lev.M @ f), scale, 1e-12, f"resid level {l}")
    s.close()
