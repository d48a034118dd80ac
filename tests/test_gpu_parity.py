"""GPU parity of the HIP solve path against the CPU oracle (FP64).

The library and the oracle each build their own hierarchy from the same
seeded inputs (they share no code); the tests compare, on the same random
vectors: every level kernel (products with A, P, R, one smoothing sweep, the
residual, the coarsest solve), one V-cycle, and whole CG solves (iteration
count within one, FP64 true residual recomputed by scipy, solution error
against a tightly converged oracle solve).  At the full 64^3 size, where the
oracle would be slow, sampled rows and size-independent properties are used.

Tolerances (FP64): level-1 products 1e-14 normwise (identical operator,
different summation order); coarser levels 1e-12 (their operators are built
independently and agree to ~1e-14); the coarsest solve uses an explicit
inverse on the GPU and a Cholesky solve in the oracle, which agree to
kappa * eps, tested at 1e-10; V-cycle 1e-11.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import meshgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_09056_amd import Solver, AmgError  # noqa: E402

from parity import assert_close, assert_close_scaled  # noqa: E402
from paper_2202_09056_amd import _capi  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = {
    "cube10": lambda: meshgen.cube_c1(10),
    "lognormal14": lambda: meshgen.cube_lognormal(14, seed=0),
    "lognormal22": lambda: meshgen.cube_lognormal(22, seed=0),
    "inclusions20": lambda: meshgen.cube_inclusions(20, n_incl=12, radius_elems=3.0),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    torch.cuda.set_device(0)
    p = CASES[request.param]()
    print(f"[case] {request.param} n={p.n} nnzb={p.nnzb}", flush=True)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords)
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    yield request.param, p, A, h, s
    s.close()


def test_hierarchy_shape_matches_oracle(case):
    name, p, A, h, s = case
    st = s.stats()
    assert st.levels == len(h.levels)
    assert [3 * st.nb[l] for l in range(st.levels)] == h.sizes()


def test_level_kernels_match_oracle(case):
    """Every entry against the rounding scale of its own row: level-1
    operators are identical (summation order only), coarser ones are built
    independently and agree to ~1e-14 relative per entry."""
    name, p, A, h, s = case
    rng = np.random.default_rng(42)
    L = len(h.levels)
    for l in range(L - 1):
        lev, nxt = h.levels[l], h.levels[l + 1]
        rel = 1e-14 if l == 0 else 1e-12
        aA, aP, aR, aM, aMt = abs(lev.A), abs(lev.P), abs(lev.R), abs(lev.M), abs(lev.Mt)
        u = rng.standard_normal(lev.n)
        v = rng.standard_normal(lev.n)
        uc = rng.standard_normal(nxt.n)
        au, av, auc = np.abs(u), np.abs(v), np.abs(uc)
        du, dv, duc = _dev(u), _dev(v), _dev(uc)
        out = torch.empty(lev.n, dtype=torch.float64, device="cuda")
        outc = torch.empty(nxt.n, dtype=torch.float64, device="cuda")
        s.debug_apply(l, 0, du, out)
        assert_close_scaled(out.cpu().numpy(), lev.A @ u, aA @ au, rel, f"A level {l}")
        s.debug_apply(l, 1, du, outc)
        assert_close_scaled(outc.cpu().numpy(), lev.R @ u, aR @ au, 1e-12, f"R level {l}")
        s.debug_apply(l, 2, duc, out)
        assert_close_scaled(out.cpu().numpy(), lev.P @ uc, aP @ auc, 1e-12, f"P level {l}")
        s.debug_apply(l, 3, du, out)
        assert_close_scaled(out.cpu().numpy(), lev.M @ u, aM @ au, 1e-12, f"M level {l}")
        s.debug_apply(l, 4, du, out, in2=dv)
        ref = v + lev.Mt @ (u - lev.A @ v)
        assert_close_scaled(out.cpu().numpy(), ref, av + aMt @ (au + aA @ av), 1e-12, f"smooth level {l}")
        s.debug_apply(l, 6, du, out, in2=dv)
        assert_close_scaled(out.cpu().numpy(), u - lev.A @ v, au + aA @ av, rel, f"resid level {l}")
        # fused sweeps: t = f - A (M f) below the first level, and on every
        # level z = P e + M (f + t) - M A P e, against the oracle's operators
        if l == 0:
            with pytest.raises(AmgError):  # level 1 keeps its own residual
                s.debug_apply(l, 11, du, out)
        else:
            s.debug_apply(l, 11, du, out)
            assert_close_scaled(out.cpu().numpy(), u - lev.A @ (lev.M @ u), au + aA @ (aM @ au), 1e-12,
                                f"fused resid level {l}")
        out.copy_(dv)
        s.debug_apply(l, 12, duc, out, in2=du)
        pe = lev.P @ uc
        ape = aP @ auc
        ref = pe - lev.M @ (lev.A @ pe) + lev.M @ (u + v)
        scale = ape + aM @ (aA @ ape) + aM @ (au + av)
        assert_close_scaled(out.cpu().numpy(), ref, scale, 1e-12, f"fused post level {l}")
    last = h.levels[-1]
    f = rng.standard_normal(last.n)
    out = torch.empty(last.n, dtype=torch.float64, device="cuda")
    s.debug_apply(0, 5, _dev(f), out)
    # explicit inverse against a Cholesky solve: kappa * u, entry by entry
    assert_close(out.cpu().numpy(), sla.cho_solve(last.chol, f), 1e-10, 1e-10, "coarsest")


def test_vcycle_matches_oracle(case):
    name, p, A, h, s = case
    rng = np.random.default_rng(7)
    r = rng.standard_normal(p.n)
    z = s.vcycle(_dev(r)).cpu().numpy()
    assert_close(z, oracle.vcycle(h, r), 1e-10, 1e-11, f"{name} V-cycle")


def test_solve_matches_oracle(case):
    name, p, A, h, s = case
    ref = oracle.amg_pcg(h, p.b, tol=1e-8, maxiter=3000)
    x, info, status = s.solve(_dev(p.b), tol=1e-8)
    xh = x.cpu().numpy()
    print(f"[solve] {name}: gpu iters={info.iters} oracle iters={ref.iters} "
          f"gpu rel={info.rel_true_residual:.3e}", flush=True)
    assert status == _capi.AMG_OK and info.converged == 1
    assert oracle.true_residual_norm(A, p.b, xh) <= 1e-8
    assert abs(info.iters - ref.iters) <= 1
    # two FP64 evaluations of ||b - A x|| / ||b|| in different summation
    # orders differ by a few units of u ||(|A| |x|)|| / ||b|| (u = 2^-53);
    # the 1000:1 inclusion case makes that term ~1e-10
    bound = 4 * 2.0 ** -53 * np.linalg.norm(abs(A) @ np.abs(xh)) / np.linalg.norm(p.b)
    assert abs(info.rel_true_residual - oracle.true_residual_norm(A, p.b, xh)) <= 1e-12 + bound
    if not name.startswith("inclusions"):
        # solution error against a direct solve; the 1000:1 inclusion case has
        # kappa ~ 1e7, where a 1e-8 residual does not bound the error by 1e-6
        exact = spla.splu(A.tocsc()).solve(p.b)
        assert _rel(xh, exact) <= 1e-6


def test_graphs_and_direct_launches_agree_bitwise():
    p = meshgen.cube_lognormal(12, seed=1)
    b = _dev(p.b)
    s1 = Solver(p.row_ptr, p.col, p.val, p.coords, use_graphs=1, check_every=4)
    s2 = Solver(p.row_ptr, p.col, p.val, p.coords, use_graphs=0, check_every=1)
    x1, i1, _ = s1.solve(b)
    x1b, i1b, _ = s1.solve(b)
    x2, i2, _ = s2.solve(b)
    assert i1.iters == i2.iters == i1b.iters
    assert torch.equal(x1, x2) and torch.equal(x1, x1b)  # deterministic reductions


def test_flexible_cg_converges():
    p = meshgen.cube_lognormal(12, seed=2)
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords, krylov="fcg")
    x, info, status = s.solve(_dev(p.b))
    assert status == 0 and oracle.true_residual_norm(A, p.b, x.cpu().numpy()) <= 1e-8
    ref = oracle.amg_pcg(oracle.build_hierarchy(A, p.coords), p.b, flexible=True)
    assert abs(info.iters - ref.iters) <= 1


def test_edge_cases():
    p = meshgen.cube_c1(10)  # two levels
    s = Solver(p.row_ptr, p.col, p.val, p.coords, maxiter=3)
    assert s.stats().levels == 2
    zero = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    x, info, status = s.solve(zero, torch.ones_like(zero))
    assert status == 0 and info.iters == 0 and not x.any()
    bad = _dev(p.b)
    bad[7] = float("nan")
    x, info, status = s.solve(bad, raise_on_error=False)
    assert status == _capi.AMG_ERR_ARG
    x, info, status = s.solve(_dev(p.b), tol=1e-12, raise_on_error=False)
    assert status == _capi.AMG_NOT_CONVERGED and info.iters == 3
    # warm start at the solution: no iteration needed
    exact = sla.solve(p.csr().toarray(), p.b, assume_a="pos")
    x, info, status = s.solve(_dev(p.b), _dev(exact), tol=1e-8)
    assert status == 0 and info.iters == 0


def test_single_level_problem_is_a_dense_solve():
    p = meshgen.cube_c1(3)  # 192 unknowns: below the coarse threshold
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    assert s.stats().levels == 1
    x, info, status = s.solve(_dev(p.b), tol=1e-10)
    exact = sla.solve(p.csr().toarray(), p.b, assume_a="pos")
    assert status == 0 and info.iters <= 2
    assert _rel(x.cpu().numpy(), exact) <= 1e-9


def test_setup_errors_are_reported():
    p = meshgen.cube_c1(4)
    val = p.val.copy()
    val[p.row_ptr[5]:p.row_ptr[6]] *= 0.0  # row 5: zero diagonal block
    with pytest.raises(AmgError):
        Solver(p.row_ptr, p.col, val, p.coords)
    with pytest.raises(AmgError):
        Solver(p.row_ptr, p.col, -p.val, p.coords)


@pytest.mark.parametrize("forced,sorted_", [(4, 0), (8, 0), (1, 0), (2, 0), (16, 0), (16, 1), (32, 1), (64, 1),
                                             (8, 1)])
def test_tune_cache_forces_layouts(forced, sorted_, tmp_path, monkeypatch):
    """Every operator's layout taken from a SAAMG_TUNE_CACHE file: the
    entries are hits (nothing is retimed or appended) and the V-cycle (entry
    by entry), the level-1 fused post-sweep and the solve agree with the
    oracle whatever the slice width and row order (sorted: rows ordered by
    length within windows, the layout of the bench's dominant kernel)."""
    p = meshgen.cube_lognormal(22, seed=0)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords)
    tuned = tmp_path / "tuned.txt"
    monkeypatch.setenv("SAAMG_TUNE_CACHE", str(tuned))
    Solver(p.row_ptr, p.col, p.val, p.coords).close()
    lines = tuned.read_text().splitlines()
    assert len(lines) >= 3
    forced_file = tmp_path / f"forced{forced}_{sorted_}.txt"
    text = "".join(" ".join(ln.split()[:4] + [str(forced), str(sorted_)]) + "\n" for ln in lines)
    forced_file.write_text(text)
    monkeypatch.setenv("SAAMG_TUNE_CACHE", str(forced_file))
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    assert forced_file.read_text() == text
    st = s.stats()
    code = -forced if (sorted_ and forced > 2) else forced
    assert st.layout_A[0] == code and st.layout_G[0] == code
    rng = np.random.default_rng(11)
    r = rng.standard_normal(p.n)
    assert_close(s.vcycle(_dev(r)).cpu().numpy(), oracle.vcycle(h, r), 1e-10, 1e-11, "V-cycle")
    lev, nxt = h.levels[0], h.levels[1]
    f, t, e = rng.standard_normal(lev.n), rng.standard_normal(lev.n), rng.standard_normal(nxt.n)
    out = _dev(t)
    s.debug_apply(0, 12, _dev(e), out, in2=_dev(f))
    pe = lev.P @ e
    ape = abs(lev.P) @ np.abs(e)
    scale = ape + abs(lev.M) @ (abs(lev.A) @ ape) + abs(lev.M) @ (np.abs(f) + np.abs(t))
    assert_close_scaled(out.cpu().numpy(), pe - lev.M @ (lev.A @ pe) + lev.M @ (f + t), scale, 1e-12,
                        "fused post-sweep, level 1")
    ref = oracle.amg_pcg(h, p.b, tol=1e-8, maxiter=3000)
    x, info, status = s.solve(_dev(p.b))
    s.close()
    print(f"[tune cache] C={forced} sorted={sorted_}: iters={info.iters} oracle={ref.iters}", flush=True)
    assert status == 0 and abs(info.iters - ref.iters) <= 1
    assert oracle.true_residual_norm(A, p.b, x.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("name,folds", [("lognormal24", True), ("cube32", False)])
def test_folded_coarsest_restriction(name, folds):
    """The last restriction is folded into the coarsest solve (one dense
    W = A_L^-1 R product per cycle) only where W streams at most about one
    launch's worth of bytes more than R and the inverse: on the 24^3 cube W is
    13.7 MB against 1.8 MB, on the 32^3 cube 31.4 MB against 3.3 MB.  Either
    way the V-cycle equals the oracle's entry by entry."""
    p = {"lognormal24": lambda: meshgen.cube_lognormal(24, seed=0), "cube32": lambda: meshgen.cube_c1(32)}[name]()
    h = oracle.build_hierarchy(p.csr(), p.coords)
    assert len(h.levels) == 3
    for prec in ("fp64", "fp32"):
        s = Solver(p.row_ptr, p.col, p.val, p.coords, precision=prec)
        if folds:
            ms, nbytes = s.time_op(0, 16, reps=2)
            assert nbytes >= h.levels[2].n * h.levels[1].n * 8
        else:
            with pytest.raises(AmgError):
                s.time_op(0, 16, reps=2)
        r = np.random.default_rng(24).standard_normal(p.n)
        got = s.vcycle(_dev(r)).cpu().numpy()
        s.close()
        ref = oracle.vcycle(h, r)
        if prec == "fp64":
            assert_close(got, ref, 1e-10, 1e-11, f"{name} V-cycle")
        else:
            assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref), name


@pytest.mark.parametrize("layout", ["tuned", "sell16_sorted"])
def test_cube40_vcycle_and_post_sweep_entrywise(layout, tmp_path, monkeypatch):
    """40^3 lognormal cube (206,763 unknowns, the largest the oracle builds
    within the test's time): the whole V-cycle and the level-1 fused
    post-sweep against the oracle entry by entry, with the tuner's layouts
    and with every operator in the bench's dominant layout (SELL-16, rows
    sorted within windows)."""
    if layout == "sell16_sorted":
        tuned = tmp_path / "tuned.txt"
        monkeypatch.setenv("SAAMG_TUNE_CACHE", str(tuned))
    p = meshgen.cube_lognormal(40, seed=0)
    print(f"[cube40] {layout} n={p.n}", flush=True)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords)
    if layout == "sell16_sorted":
        # every sparse operator of this hierarchy, forced to SELL-16 sorted
        from paper_2202_09056_amd import HostHierarchy
        H = HostHierarchy(p.row_ptr, p.col, p.val, p.coords)
        keys = []
        for l in range(H.levels - 1):
            for op in ("A", "P", "R", "AM", "G"):
                rp, col, _, (rows, cols) = H.bsr(l, op)
                if col.size:
                    keys.append(f"{rows} {cols} {col.size} 8 16 1")
        H.close()
        tuned.write_text("\n".join(keys) + "\n")
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    if layout == "sell16_sorted":
        st = s.stats()
        assert st.layout_G[0] == -16 and st.layout_A[0] == -16
    rng = np.random.default_rng(40)
    r = rng.standard_normal(p.n)
    assert_close(s.vcycle(_dev(r)).cpu().numpy(), oracle.vcycle(h, r), 1e-10, 1e-11, "V-cycle 40^3")
    lev, nxt = h.levels[0], h.levels[1]
    f, t, e = rng.standard_normal(lev.n), rng.standard_normal(lev.n), rng.standard_normal(nxt.n)
    out = _dev(t)
    s.debug_apply(0, 12, _dev(e), out, in2=_dev(f))
    s.close()
    pe = lev.P @ e
    ape = abs(lev.P) @ np.abs(e)
    scale = ape + abs(lev.M) @ (abs(lev.A) @ ape) + abs(lev.M) @ (np.abs(f) + np.abs(t))
    assert_close_scaled(out.cpu().numpy(), pe - lev.M @ (lev.A @ pe) + lev.M @ (f + t), scale, 1e-12,
                        "fused post-sweep, level 1, 40^3")


@pytest.mark.parametrize("n", [64])
def test_full_size_lognormal_cube(n):
    """64^3 lognormal cube: sampled rows of A x, V-cycle symmetry and
    positivity, and the FP64 true residual of the solve (scipy)."""
    p = meshgen.cube_lognormal(n, seed=0)
    print(f"[full] cube{n} lognormal n={p.n}", flush=True)
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(p.n)
    v = rng.standard_normal(p.n)
    out = torch.empty(p.n, dtype=torch.float64, device="cuda")
    s.debug_apply(0, 0, _dev(u), out)
    rows = rng.choice(p.n, 2000, replace=False)
    ref = A[rows] @ u
    got = out.cpu().numpy()[rows]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    Vu = s.vcycle(_dev(u)).cpu().numpy()
    Vv = s.vcycle(_dev(v)).cpu().numpy()
    assert abs(v @ Vu - u @ Vv) <= 1e-11 * abs(v @ Vu)
    assert u @ Vu > 0 and v @ Vv > 0
    x, info, status = s.solve(_dev(p.b), tol=1e-8)
    rel = oracle.true_residual_norm(A, p.b, x.cpu().numpy())
    print(f"[full] iters={info.iters} rel={rel:.3e} ms={info.solve_ms:.1f}", flush=True)
    assert status == 0 and rel <= 1e-8
