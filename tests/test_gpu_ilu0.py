"""GPU parity of the block ILU(0) smoother in multicolour order (Section 3:
ILU(0) with 3x3 block values, the smoother of the paper's experiments;
Section 4 and Tables 1-2).

The library and the oracle factor their own hierarchies from the same
inputs.  FP64: one application of (L U)^{-1}, one smoothing sweep and the
whole V-cycle agree with the oracle entry by entry (the factors differ only
in rounding; the triangular solves run one pass per colour on the device and
as scalar triangular solves in the oracle), and CG takes the oracle's
iteration count within one, with ILU(0) on the first level (block Jacobi
below) and on every level.  The FP32 V-cycle stays within FP32 rounding of
the FP64 one and its solve reaches the FP64 true residual 1e-8.
"""
import numpy as np
import pytest

import meshgen
import oracle

from parity import assert_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_09056_amd import Solver, BatchSolver, AmgError  # noqa: E402
from paper_2202_09056_amd import _capi  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


CASES = {
    "cube10": lambda: (meshgen.cube_c1(10), {}),
    "lognormal14": lambda: (meshgen.cube_lognormal(14, seed=0), {}),
    "tets12": lambda: (meshgen.tet_cube(12), {}),
    "lognormal16_3lvl_l1": lambda: (meshgen.cube_lognormal(16, seed=1), {"coarse_enough": 300}),
    "lognormal16_3lvl_all": lambda: (meshgen.cube_lognormal(16, seed=1), {"coarse_enough": 300,
                                                                          "smoother_levels": 0}),
}


def _hierarchies(name):
    p, kw = CASES[name]()
    okw = dict(kw)
    lv = okw.pop("smoother_levels", 1)
    h = oracle.build_hierarchy(p.csr(), p.coords,
                               oracle.AmgParams(smoother="ilu0_mc", smoother_levels=lv or None, **okw))
    return p, kw, h


@pytest.mark.parametrize("name", list(CASES))
def test_ilu0_vcycle_and_solve_match_oracle(name):
    p, kw, h = _hierarchies(name)
    print(f"[ilu0] {name} n={p.n} levels={len(h.levels)}", flush=True)
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="ilu0", **kw)
    assert s.stats().levels == len(h.levels)
    rng = np.random.default_rng(11)
    r = rng.standard_normal(p.n)
    assert_close(s.vcycle(_dev(r)).cpu().numpy(), oracle.vcycle(h, r), 1e-10, 1e-12, f"{name} V-cycle")
    ref = oracle.amg_pcg(h, p.b, tol=1e-8, maxiter=3000)
    x, info, status = s.solve(_dev(p.b), tol=1e-8)
    s.close()
    print(f"[ilu0] {name}: gpu iters={info.iters} oracle iters={ref.iters}", flush=True)
    assert status == _capi.AMG_OK and info.converged == 1
    assert abs(info.iters - ref.iters) <= 1
    assert oracle.true_residual_norm(A, p.b, x.cpu().numpy()) <= 1e-8


def test_ilu0_single_sweeps_match_oracle_on_every_ilu_level():
    """op 3: (L U)^{-1} f; op 4: x + (L U)^{-1} (f - A x), on each level of a
    three-level hierarchy with ILU(0) everywhere."""
    p, kw, h = _hierarchies("lognormal16_3lvl_all")
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="ilu0", **kw)
    rng = np.random.default_rng(5)
    for l in range(len(h.levels) - 1):
        lev = h.levels[l]
        f, x = rng.standard_normal(lev.n), rng.standard_normal(lev.n)
        out = _dev(np.zeros(lev.n))
        s.debug_apply(l, 3, _dev(f), out)
        assert_close(out.cpu().numpy(), lev.M @ f, 1e-10, 1e-12, f"(LU)^-1 f level {l}")
        s.debug_apply(l, 4, _dev(f), out, in2=_dev(x))
        assert_close(out.cpu().numpy(), x + lev.M @ (f - lev.A @ x), 1e-10, 1e-12, f"sweep level {l}")
    s.close()


def test_ilu0_vcycle_is_symmetric():
    # L U = L D L^T for symmetric A: the same operator before and after the
    # coarse correction gives a symmetric V-cycle
    p = meshgen.cube_lognormal(12, seed=2)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="ilu0", coarse_enough=300, smoother_levels=0)
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(p.n), rng.standard_normal(p.n)
    va = s.vcycle(_dev(a)).cpu().numpy()
    vb = s.vcycle(_dev(b)).cpu().numpy()
    s.close()
    assert abs(va @ b - a @ vb) <= 1e-11 * np.linalg.norm(va) * np.linalg.norm(b)


def test_ilu0_fp32_vcycle_and_solve():
    p, kw, h = _hierarchies("lognormal14")
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="ilu0", precision="fp32")
    rng = np.random.default_rng(8)
    r = rng.standard_normal(p.n)
    z = s.vcycle(_dev(r)).cpu().numpy()
    ref = oracle.vcycle(h, r)
    assert np.linalg.norm(z - ref) <= 1e-4 * np.linalg.norm(ref)
    x, info, status = s.solve(_dev(p.b), tol=1e-8)
    s.close()
    assert status == _capi.AMG_OK and info.converged == 1
    assert oracle.true_residual_norm(A, p.b, x.cpu().numpy()) <= 1e-8


def test_ilu0_cuts_iterations_against_block_jacobi():
    p = meshgen.cube_lognormal(16, seed=0)
    its = {}
    for sm in ("jacobi", "ilu0"):
        s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother=sm, coarse_enough=300)
        _, info, status = s.solve(_dev(p.b), tol=1e-8)
        s.close()
        assert status == _capi.AMG_OK
        its[sm] = info.iters
    assert its["ilu0"] < its["jacobi"], its


def test_ilu0_rejected_by_multi_rhs_and_batch():
    p = meshgen.cube_c1(6)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="ilu0", coarse_enough=100)
    B = _dev(np.zeros((p.n, 2)))
    with pytest.raises(AmgError):
        s.solve_multi(B)
    s.close()
    with pytest.raises(AmgError):
        BatchSolver([(p.row_ptr, p.col, p.val, p.coords)], smoother="ilu0")
