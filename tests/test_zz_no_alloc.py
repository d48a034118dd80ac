"""The entry point that allocates nothing (amg_true_residual_noalloc): its
scratch -- partial sums and reduction state -- lives in a static device array
instead of context memory.  Checked against amg_true_residual, the entry
point it varies, on two calls in a row with the second on a smaller problem
(whose launch uses fewer partial sums than the first left in the array), and
r = b - A x against the oracle's matrix entry by entry."""
import numpy as np
import pytest

import meshgen

from parity import assert_close_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_09056_amd import Solver, AmgError  # noqa: E402
from paper_2202_09056_amd import _capi  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _check(p, seed):
    A = p.csr()
    rng = np.random.default_rng(seed)
    b, x = rng.standard_normal(p.n), rng.standard_normal(p.n)
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    db, dx = _dev(b), _dev(x)
    ref_rel = s.true_residual(db, dx)
    r = torch.full((p.n,), np.nan, dtype=torch.float64, device="cuda")
    norms = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    rel = s.true_residual_noalloc(db, dx, r, norms)
    assert rel == ref_rel  # same kernels, same partial sums, same order
    nb, nr = norms.cpu().numpy()
    assert np.sqrt(nr / nb) == rel
    assert abs(nb - b @ b) <= 1e-13 * (b @ b)
    scale = abs(A) @ np.abs(x) + np.abs(b)
    assert_close_rows(r.cpu().numpy(), b - A @ x, scale, 2 * (1 + A.getnnz(axis=1).max()), "r = b - A x")
    # the asynchronous form leaves the same norms once the stream is done
    norms2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    assert s.true_residual_noalloc(db, dx, r, norms2, sync=False) is None
    torch.cuda.synchronize()
    assert torch.equal(norms2, norms)
    s.close()
    return ref_rel


def test_noalloc_true_residual_matches_allocating_entry_point():
    big = meshgen.cube_lognormal(20, seed=0)     # first call: more partial sums
    small = meshgen.cube_c1(7)                   # second call: fewer, on a fresh context
    print(f"[noalloc] n={big.n} then n={small.n}", flush=True)
    r1 = _check(big, 1)
    r2 = _check(small, 2)
    assert r1 > 0 and r2 > 0


def test_noalloc_rejects_bad_arguments():
    p = meshgen.cube_c1(5)
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    b = _dev(np.ones(p.n))
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(AmgError):
        s.true_residual_noalloc(b, b.clone(), b, norms)  # r aliases b
    s.close()


def test_noalloc_rejects_a_launch_beyond_the_scratch(tmp_path, monkeypatch):
    """A finest operator forced to one workgroup per block row (layout code 2)
    with more block rows than the static array holds partial sums for."""
    p = meshgen.cube_c1(41)  # 42^3 = 74,088 block rows
    cap = ((1 << 20) - 256) // 16
    assert p.nb > cap
    nnzb = int(p.row_ptr[-1])
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{p.nb} {p.nb} {nnzb} 8 2 0\n")
    monkeypatch.setenv("SAAMG_TUNE_CACHE", str(cache))
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    assert s.stats().layout_A[0] == 2
    b = _dev(np.ones(p.n))
    r = torch.empty_like(b)
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(AmgError, match="static scratch"):
        s.true_residual_noalloc(b, b.clone(), r, norms)
    # the allocating entry point still handles it
    assert s.true_residual(b, torch.zeros_like(b)) == pytest.approx(1.0, rel=1e-15)
    s.close()
