"""Pins of the oracle's learned smoother blocks (CPU).

Each check is fixed by something other than the oracle's own formulas:
grid indices for the slots, the similarity M^{-1} S ~ I + X for a network
with a known constant output, generalised eigenvalues for the band, the
energy contraction it implies, central finite differences for the gradient,
Adam's first step in closed form, and block Jacobi for a zero output layer.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import meshgen
import oracle
from oracle import learned as OL


def _beam_level(nx=8, ny=2, coarse_enough=100):
    p = meshgen.beam(nx, ny, ny)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords, oracle.AmgParams(coarse_enough=coarse_enough))
    return p, A, h, OL.learned_level(h, p.row_ptr, p.col, p.val, p.coords)


def _random_theta(rng, scale=0.3):
    return rng.standard_normal(OL.N_PARAMS) * scale


def test_parameter_count():
    assert OL.N_PARAMS == 90 * 64 + 64 + 64 * 64 + 64 + 64 * 6 + 6 == 10374


def test_slots_follow_grid_offsets():
    nx, ny, nz = 3, 2, 2
    p = meshgen.assemble_box(nx, ny, nz, 0.5, 0.25, 0.25, 0.3, None, clamp_x0=False)
    row_ptr, col, coords = p[0], p[1], p[3]
    slots = OL.neighbour_slots(row_ptr, col, coords)
    # node index -> grid position, from the generator's x-fastest numbering
    nnx, nny = nx + 1, ny + 1
    def pos(i):
        return np.array([i % nnx, (i // nnx) % nny, i // (nnx * nny)])
    k = 0
    for i in range(row_ptr.shape[0] - 1):
        for kk in range(row_ptr[i], row_ptr[i + 1]):
            d = pos(col[kk]) - pos(i)
            assert slots[kk] == 9 * (d[0] + 1) + 3 * (d[1] + 1) + (d[2] + 1)
            k += 1
    assert k == slots.shape[0]


def test_slot_collision_rejected():
    row_ptr = np.array([0, 3, 4, 5])
    col = np.array([0, 1, 2, 1, 2])
    coords = np.array([[0.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0]])   # nodes 1 and 2 coincide
    with pytest.raises(ValueError):
        OL.neighbour_slots(row_ptr, col, coords)


def test_features_scale_free_and_symmetric():
    p, A, h, L = _beam_level()
    phi = L.phi
    assert np.allclose((phi[:, :9] ** 2).sum(axis=1), 1.0)
    # scaling A scales nothing
    phi2 = OL.features(p.row_ptr, p.col, 7.5 * p.val, p.coords)
    assert np.allclose(phi, phi2, rtol=1e-14, atol=0)
    # an interior node of a uniform grid sees the same coupling at opposite slots
    lens = np.diff(p.row_ptr)
    i = int(np.argmax(lens == 27))
    r = phi[i, 9:].reshape(27, 3)
    assert np.allclose(r, r[::-1], rtol=1e-12, atol=1e-14)


def test_zero_output_layer_is_block_jacobi():
    p, A, h, L = _beam_level()
    rng = np.random.default_rng(0)
    theta = _random_theta(rng)
    P = OL.unpack(theta)
    P["W3"][:] = 0.0
    P["b3"][:] = 0.0
    S = OL.smoother_blocks(L, theta)
    assert np.allclose(S, L.Mblk, rtol=1e-14, atol=1e-15)
    f = rng.standard_normal(p.n)
    assert np.allclose(OL.vcycle_blocks(h, S, f), oracle.vcycle(h, f), rtol=1e-12, atol=1e-14)


def test_known_constant_output():
    p, A, h, L = _beam_level()
    theta = np.zeros(OL.N_PARAMS)
    P = OL.unpack(theta)
    P["b1"][0] = 1.0           # h1 = e_0 for every node
    P["b2"][0] = 1.0           # h2 = e_0
    u = np.array([0.7, -1.3, 2.0, 0.4, -0.9, 1.1])
    P["W3"][0] = u             # g = u
    S = OL.smoother_blocks(L, theta)
    t = np.tanh(u)
    c = OL.SPREAD
    X = np.array([[c[0] * t[0], c[3] * t[3], c[4] * t[4]],
                  [c[3] * t[3], c[1] * t[1], c[5] * t[5]],
                  [c[4] * t[4], c[5] * t[5], c[2] * t[2]]])
    want = np.sort(np.linalg.eigvalsh(np.eye(3) + X))
    for i in [0, 5, L.nb // 2, L.nb - 1]:
        got = np.sort(np.linalg.eigvals(np.linalg.solve(L.Mblk[i], S[i])).real)
        assert np.allclose(got, want, rtol=1e-12), i
        assert np.allclose(S[i], S[i].T, rtol=1e-14, atol=1e-16)


def test_band_holds_for_any_output():
    p, A, h, L = _beam_level()
    rng = np.random.default_rng(1)
    theta = _random_theta(rng, scale=5.0)         # saturates tanh
    S = OL.smoother_blocks(L, theta)
    for i in range(0, L.nb, 7):
        mu = sla.eigh(S[i], L.Mblk[i], eigvals_only=True)
        assert mu.min() > 0.65 - 1e-12 and mu.max() < 1.35 + 1e-12
    assert OL.in_band(L, S).all()
    # the band makes every relaxation an energy-norm contraction
    for _ in range(5):
        e = rng.standard_normal(p.n)
        w = e - OL.block_apply(S, A @ e)
        assert w @ (A @ w) < e @ (A @ e)


def test_learned_vcycle_is_symmetric():
    p, A, h, L = _beam_level(4, 2, coarse_enough=60)
    rng = np.random.default_rng(2)
    S = OL.smoother_blocks(L, _random_theta(rng, 1.0))
    n = p.n
    B = np.column_stack([OL.vcycle_blocks(h, S, np.eye(n)[:, j]) for j in range(n)])
    assert np.allclose(B, B.T, rtol=0, atol=1e-10 * np.abs(B).max())
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_gradient_matches_central_differences():
    p, A, h, L = _beam_level(8, 2, coarse_enough=60)
    rng = np.random.default_rng(3)
    theta = _random_theta(rng, 0.4)
    E = rng.standard_normal((p.n, 2)) * meshgen_free(p)[:, None]
    loss, grad = OL.loss_and_grad(h, L, theta, E)
    assert 0.0 < loss < 1.0
    starts = {name: o for name, o in zip([n for n, _ in OL.SHAPES],
                                          np.cumsum([0] + [int(np.prod(s)) for _, s in OL.SHAPES]))}
    picks = [starts["W1"] + 9 * 64 + 3, starts["W1"] + 60 * 64 + 17, starts["b1"] + 5, starts["W2"] + 7 * 64 + 40,
             starts["b2"] + 11, starts["W3"] + 2 * 6 + 1, starts["W3"] + 40 * 6 + 5, starts["b3"] + 0,
             starts["b3"] + 4]
    hstep = 1e-5
    for k in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += hstep
        tm[k] -= hstep
        fd = (OL.loss_only(h, L, tp, E) - OL.loss_only(h, L, tm, E)) / (2 * hstep)
        assert abs(fd - grad[k]) <= 1e-5 * max(1e-3, abs(grad[k])) + 1e-9, (k, fd, grad[k])


def meshgen_free(p):
    return np.repeat(~p.fixed, 3).astype(float)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = OL.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-8)
    assert np.allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_errors_are_stationary_iterates():
    p, A, h, L = _beam_level()
    rng = np.random.default_rng(5)
    e0 = rng.standard_normal(p.n)
    E = OL.training_errors(h, e0, cycles=2)
    # e - V(A e) is the error of x + V(b - A x) for b = A x*, x* - x = e
    xs = rng.standard_normal(p.n)
    b = A @ xs
    x = xs - e0
    for _ in range(2):
        x = x + oracle.vcycle(h, b - A @ x)
    assert np.allclose(E[:, 0], xs - x, rtol=1e-10, atol=1e-12)
