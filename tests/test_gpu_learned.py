"""GPU checks of the learned level-1 smoother blocks.

Against the FP64 oracle on the same seeded inputs: the installed blocks S(theta)
(network in FP32 on the GPU), the training errors, the two-grid loss and its
gradient (GPU forward/backward kernels vs the oracle's NumPy reference,
itself pinned by central differences), and whole solves with the learned
blocks.  Then the fallback paths, and the gain test: a network trained by the
library's kernels on small beams against block Jacobi on a held-out beam
(the gain is measured, parity unpinned).
"""
import numpy as np
import pytest

import meshgen
import oracle
from oracle import learned as OL

from parity import assert_close, assert_close_scaled

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_09056_amd import Solver, _capi  # noqa: E402
from paper_2202_09056_amd import learned as LD  # noqa: E402


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _theta(seed, scale=0.3):
    return np.random.default_rng(seed).standard_normal(OL.N_PARAMS) * scale


def _dev32(theta):
    return torch.from_numpy(np.asarray(theta, dtype=np.float32)).cuda()


@pytest.fixture(scope="module", params=["beam32x4x4", "beam64x8x8"])
def case(request):
    nx, ny = {"beam32x4x4": (32, 4), "beam64x8x8": (64, 8)}[request.param]
    p = meshgen.beam(nx, ny, ny)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords, oracle.AmgParams(coarse_enough=500))
    L = OL.learned_level(h, p.row_ptr, p.col, p.val, p.coords)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="learned", coarse_enough=500)
    print(f"[learned] case {request.param}: levels {h.sizes()}", flush=True)
    yield request.param, p, A, h, L, s
    s.close()


def test_installed_blocks_match_oracle(case):
    name, p, A, h, L, s = case
    theta = _theta(11, 0.5)
    # the oracle evaluates the network on the FP32-rounded weights the GPU uses
    theta32 = np.asarray(theta, dtype=np.float32).astype(np.float64)
    assert s.set_smoother_weights(_dev32(theta)) == 0
    S = OL.smoother_blocks(L, theta32)
    u = np.random.default_rng(12).standard_normal(p.n)
    out = torch.empty(p.n, dtype=torch.float64, device="cuda")
    s.debug_apply(0, 3, torch.from_numpy(u).cuda(), out)
    err = _rel(out.cpu().numpy(), OL.block_apply(S, u))
    print(f"[learned] {name}: S u vs oracle {err:.2e}", flush=True)
    assert err <= 1e-5
    # block Jacobi again
    s.set_smoother_weights(None)
    s.debug_apply(0, 3, torch.from_numpy(u).cuda(), out)
    assert_close_scaled(out.cpu().numpy(), h.levels[0].M @ u, abs(h.levels[0].M) @ np.abs(u), 1e-14, "M")


def test_bf16_weights_equal_fp32_of_the_rounded_values(case):
    """BF16 parameters are widened to FP32 exactly before the forward pass, so
    the installed blocks are bit-for-bit those of the FP32 tensor holding the
    same rounded values; the C ABI rejects a byte count or type that does not
    match."""
    import ctypes as C
    name, p, A, h, L, s = case
    t16 = torch.from_numpy(_theta(21, 0.5).astype(np.float32)).to(torch.bfloat16).cuda()
    t32 = t16.float()
    u = torch.from_numpy(np.random.default_rng(22).standard_normal(p.n)).cuda()
    out16 = torch.empty(p.n, dtype=torch.float64, device="cuda")
    out32 = torch.empty_like(out16)
    assert s.set_smoother_weights(t16) == 0
    s.debug_apply(0, 3, u, out16)
    assert s.set_smoother_weights(t32) == 0
    s.debug_apply(0, 3, u, out32)
    assert torch.equal(out16, out32)
    S = OL.smoother_blocks(L, t32.cpu().double().numpy())
    assert _rel(out16.cpu().numpy(), OL.block_apply(S, u.cpu().numpy())) <= 1e-5
    lib = _capi.load()
    nbad = C.c_int32(0)
    bf16, fp64 = _capi.PRECISIONS["bf16"], _capi.PRECISIONS["fp64"]
    for nbytes, dtype in [(4 * OL.N_PARAMS, bf16), (2 * OL.N_PARAMS - 2, bf16), (8 * OL.N_PARAMS, fp64)]:
        st = lib.amg_smoother_set_weights(s.ctx, C.c_void_p(t16.data_ptr()), nbytes, dtype, 1, C.byref(nbad))
        assert st == _capi.AMG_ERR_ARG, (nbytes, dtype)
    with pytest.raises(TypeError):
        s.set_smoother_weights(t32.double())
    s.set_smoother_weights(None)


def test_vcycle_follows_installed_blocks(case):
    """The level-1 post-sweep operator G = (I - S A) P is formed again on the
    device whenever blocks are installed or restored: the V-cycle matches the
    oracle's with the learned blocks, then with block Jacobi again, and after a
    loss evaluation (which installs blocks without rebuilding G) a V-cycle
    still uses the blocks in place."""
    name, p, A, h, L, s = case
    theta = _theta(13, 0.5)
    theta32 = np.asarray(theta, dtype=np.float32).astype(np.float64)
    r = np.random.default_rng(14).standard_normal(p.n)
    s.set_smoother_weights(_dev32(theta))
    got = s.vcycle(torch.from_numpy(r).cuda()).cpu().numpy()
    ref = OL.vcycle_blocks(h, OL.smoother_blocks(L, theta32), r)
    err = _rel(got, ref)
    print(f"[learned] {name}: learned V-cycle vs oracle {err:.2e}", flush=True)
    assert err <= 1e-5
    s.set_smoother_weights(None)
    assert_close(s.vcycle(torch.from_numpy(r).cuda()).cpu().numpy(), oracle.vcycle(h, r), 1e-10, 1e-11, "V-cycle")
    E0 = np.random.default_rng(15).standard_normal((2, p.n))
    grad = torch.zeros(OL.N_PARAMS, dtype=torch.float32, device="cuda")
    s.mlp_loss_grad(_dev32(theta), torch.from_numpy(E0).cuda(), grad)   # installs S(theta)
    assert _rel(s.vcycle(torch.from_numpy(r).cuda()).cpu().numpy(), ref) <= 1e-5
    s.set_smoother_weights(None)


def test_training_errors_match_oracle(case):
    name, p, A, h, L, s = case
    s.set_smoother_weights(None)
    E0 = np.random.default_rng(13).standard_normal((3, p.n)) * LD.free_mask(p.row_ptr)
    E = torch.from_numpy(E0).cuda()
    s.training_errors(E, 2)
    ref = OL.training_errors(h, E0.T, 2)
    err = _rel(E.cpu().numpy(), ref.T)
    assert err <= 1e-11, err


def test_loss_and_gradient_match_oracle(case):
    name, p, A, h, L, s = case
    theta = np.asarray(_theta(14, 0.4), dtype=np.float32).astype(np.float64)
    rng = np.random.default_rng(15)
    E0 = rng.standard_normal((3, p.n)) * LD.free_mask(p.row_ptr)
    grad = torch.zeros(OL.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = s.mlp_loss_grad(_dev32(theta), torch.from_numpy(E0).cuda(), grad)
    ref_loss, ref_grad = OL.loss_and_grad(h, L, theta, E0.T)
    g = grad.cpu().numpy().astype(np.float64)
    err = _rel(g, ref_grad)
    print(f"[learned] {name}: loss {loss:.6f} (oracle {ref_loss:.6f}), gradient rel. error {err:.2e}", flush=True)
    assert abs(loss - ref_loss) <= 1e-6 * abs(ref_loss)
    assert err <= 1e-4
    # per layer, so a small layer cannot hide behind a large one
    o = 0
    for lname, shape in OL.SHAPES:
        k = int(np.prod(shape))
        assert _rel(g[o:o + k], ref_grad[o:o + k]) <= 1e-3, lname
        o += k
    # accumulate and scale
    loss2 = s.mlp_loss_grad(_dev32(theta), torch.from_numpy(E0).cuda(), grad, scale=0.5, accumulate=True)
    assert loss2 == loss
    assert _rel(grad.cpu().numpy().astype(np.float64), 1.5 * g) <= 1e-6


def test_adam_matches_oracle():
    p = meshgen.beam(32, 4, 4)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="learned", coarse_enough=500)
    rng = np.random.default_rng(16)
    th = rng.standard_normal(OL.N_PARAMS).astype(np.float32)
    m = np.zeros(OL.N_PARAMS)
    v = np.zeros(OL.N_PARAMS)
    T, M, Vv = _dev32(th), torch.zeros(OL.N_PARAMS, device="cuda"), torch.zeros(OL.N_PARAMS, device="cuda")
    ref = th.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(OL.N_PARAMS).astype(np.float32)
        s.mlp_adam(T, _dev32(g), M, Vv, step, 1e-2)
        ref, m, v = OL.adam_step(ref, g.astype(np.float64), m, v, step, 1e-2)
    assert _rel(T.cpu().numpy().astype(np.float64), ref) <= 1e-6
    s.close()


@pytest.mark.parametrize("name", ["cube10", "lognormal14"])
def test_learned_solve_matches_oracle(name):
    # cubes: the slender beams' FP64 residual floor sits near 1e-8
    p = {"cube10": lambda: meshgen.cube_c1(10), "lognormal14": lambda: meshgen.cube_lognormal(14, seed=0)}[name]()
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords)
    L = OL.learned_level(h, p.row_ptr, p.col, p.val, p.coords)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="learned")
    theta = np.asarray(_theta(17, 0.3), dtype=np.float32).astype(np.float64)
    s.set_smoother_weights(_dev32(theta))
    x, info, status = s.solve(torch.from_numpy(np.ascontiguousarray(p.b)).cuda(), tol=1e-8,
                              raise_on_error=False)
    S = OL.smoother_blocks(L, theta)
    ref = oracle.pcg(A, p.b, lambda r: OL.vcycle_blocks(h, S, r), tol=1e-8, maxiter=3000)
    xh = x.cpu().numpy()
    print(f"[learned] {name}: iters {info.iters} (oracle {ref.iters}), status {status}", flush=True)
    assert status == _capi.AMG_OK and info.converged == 1 and info.fell_back == 0
    assert oracle.true_residual_norm(A, p.b, xh) <= 1e-8
    assert abs(info.iters - ref.iters) <= 1
    s.close()


def test_nonfinite_weights_fall_back():
    p = meshgen.cube_lognormal(14, seed=0)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="learned")
    b = torch.from_numpy(np.ascontiguousarray(p.b)).cuda()
    _, ref, _ = s.solve(b, tol=1e-8)
    bad = _theta(18)
    bad[OL.N_PARAMS - 3] = np.nan            # an output bias: every block non-finite
    nb = p.n // 3
    assert s.set_smoother_weights(_dev32(bad), check=True) == nb    # all nodes keep M_i
    _, info, status = s.solve(b, tol=1e-8)
    assert status == 0 and info.iters == ref.iters and info.fell_back == 0
    s.set_smoother_weights(_dev32(bad), check=False)                # stored as computed
    x, info, status = s.solve(b, tol=1e-8)
    print(f"[learned] fallback: iters {info.iters} (block Jacobi {ref.iters}), fell_back {info.fell_back}",
          flush=True)
    assert status == 0 and info.converged == 1 and info.fell_back == 1
    assert oracle.true_residual_norm(p.csr(), p.b, x.cpu().numpy()) <= 1e-8
    s.close()


def test_setup_errors():
    p = meshgen.beam(32, 4, 4)
    s = Solver(p.row_ptr, p.col, p.val, p.coords, coarse_enough=500)    # block Jacobi only
    with pytest.raises(_capi.AmgError) as e:
        s.set_smoother_weights(_dev32(_theta(19)))
    assert e.value.status == _capi.AMG_ERR_UNSUPPORTED
    s.close()
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="learned", precision="fp32", coarse_enough=500)
    grad = torch.zeros(OL.N_PARAMS, dtype=torch.float32, device="cuda")
    E = torch.zeros((1, p.n), dtype=torch.float64, device="cuda")
    with pytest.raises(_capi.AmgError) as e:
        s.mlp_loss_grad(_dev32(_theta(19)), E, grad)
    assert e.value.status == _capi.AMG_ERR_UNSUPPORTED
    s.close()


def _energy_after_cycles(s, A, E0, cycles):
    """Mean e^T A e / e0^T A e0 after `cycles` stationary V-cycle steps."""
    E = torch.from_numpy(E0).cuda()
    s.training_errors(E, cycles)
    Eh = E.cpu().numpy()
    return float(np.mean([(Eh[j] @ (A @ Eh[j])) / (E0[j] @ (A @ E0[j])) for j in range(E0.shape[0])]))


def test_trained_blocks_gain_over_block_jacobi():
    """Train with the library's kernels on two small beams, then compare with
    block Jacobi on a held-out beam.  A single CG iteration count on this
    ill-conditioned beam moves by several percent with summation order alone,
    so the comparison uses the stationary V-cycle (error energy after 10
    cycles) and the mean CG iteration count over 8 random loads."""
    train = [meshgen.beam(32, 4, 4), meshgen.beam(64, 8, 8)]
    res = LD.train_smoother([(q.row_ptr, q.col, q.val, q.coords) for q in train],
                            LD.TrainConfig(steps=150), log=lambda m: print("[learned] " + m, flush=True))
    assert np.isfinite(res.theta).all()
    assert np.mean(res.losses[-20:]) < 0.97 * res.losses[0]
    # the beam's FP64 true-residual floor is near 1e-7: stop on the CG recurrence
    p = meshgen.beam(96, 12, 12)
    A = p.csr()
    s = Solver(p.row_ptr, p.col, p.val, p.coords, smoother="learned", maxiter=3000, accept_recurrence=1)
    rng = np.random.default_rng(20)
    mask = LD.free_mask(p.row_ptr)
    E0 = rng.standard_normal((4, p.n)) * mask
    B = torch.from_numpy(np.ascontiguousarray(rng.standard_normal((p.n, 8)) * mask[:, None])).cuda()
    out = {}
    for name, theta in [("block Jacobi", None), ("learned", _dev32(res.theta))]:
        s.set_smoother_weights(theta)
        energy = _energy_after_cycles(s, A, E0, 10)
        X, infos, status = s.solve_multi(B, tol=1e-8)
        assert status == 0 and all(i.converged in (1, 2) for i in infos)
        Xh, Bh = X.cpu().numpy(), B.cpu().numpy()
        worst = max(oracle.true_residual_norm(A, Bh[:, j], Xh[:, j]) for j in range(8))
        assert worst <= 1e-6
        out[name] = (energy, float(np.mean([i.iters for i in infos])))
    print(f"[learned] held-out beam96x12x12: energy after 10 V-cycles {out['block Jacobi'][0]:.3e} -> "
          f"{out['learned'][0]:.3e}; mean CG iterations over 8 loads {out['block Jacobi'][1]:.1f} -> "
          f"{out['learned'][1]:.1f}; training {res.seconds:.1f} s", flush=True)
    assert out["learned"][0] < 0.8 * out["block Jacobi"][0]
    assert out["learned"][1] < out["block Jacobi"][1]
    s.close()
