"""GPU parity on Kuhn-split P1 tetrahedral meshes (the element type of the
paper's rod and hook, Section 4): 15 block columns per row instead of the
bricks' 27, and a different aggregate shape.  The library and the oracle
build their own hierarchies from the same inputs; the FP64 V-cycle agrees to
1e-11 and CG takes the oracle's iteration count within one, with and without
the rigid body modes.  The FP32 V-cycle inside FP64 CG reaches the FP64 true
residual 1e-8.
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

from paper_2202_09056_amd import Solver  # noqa: E402
from paper_2202_09056_amd import _capi  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = {
    "tets14": lambda: (meshgen.tet_cube(14), {}),
    "tets20_3lvl": lambda: (meshgen.tet_cube(20), {"coarse_enough": 300}),
    "tets16_no_nullspace": lambda: (meshgen.tet_cube(16), {"use_nullspace": 0}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_tet_vcycle_and_solve_match_oracle(name):
    p, kw = CASES[name]()
    print(f"[tets] {name} n={p.n}", flush=True)
    A = p.csr()
    okw = dict(kw)
    if "use_nullspace" in okw:
        okw["use_nullspace"] = bool(okw["use_nullspace"])
    h = oracle.build_hierarchy(A, p.coords, oracle.AmgParams(**okw))
    s = Solver(p.row_ptr, p.col, p.val, p.coords, **kw)
    assert s.stats().levels == len(h.levels)
    rng = np.random.default_rng(8)
    r = rng.standard_normal(p.n)
    assert_close(s.vcycle(_dev(r)).cpu().numpy(), oracle.vcycle(h, r), 1e-10, 1e-11, "V-cycle")
    ref = oracle.amg_pcg(h, p.b, tol=1e-8, maxiter=3000)
    x, info, status = s.solve(_dev(p.b), tol=1e-8)
    s.close()
    print(f"[tets] {name}: gpu iters={info.iters} oracle iters={ref.iters}", flush=True)
    assert status == _capi.AMG_OK and info.converged == 1
    assert abs(info.iters - ref.iters) <= 1
    assert oracle.true_residual_norm(A, p.b, x.cpu().numpy()) <= 1e-8


def test_tet_fp32_vcycle_converges():
    p = meshgen.tet_cube(18)
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords, precision="fp32")
    x, info, status = s.solve(_dev(p.b), tol=1e-8)
    s.close()
    assert status == _capi.AMG_OK and info.converged == 1
    assert oracle.true_residual_norm(A, p.b, x.cpu().numpy()) <= 1e-8
