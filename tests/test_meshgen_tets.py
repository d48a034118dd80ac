"""Pins of the Kuhn-split P1 tetrahedral generator (the stand-ins for the
paper's connecting rod and solid hook, Section 4).

The element matrix is checked against closed forms: a linear displacement
field u(x) = G x has the constant strain eps = sym(G), so its exact strain
energy over a tetrahedron of volume V is V (lam/2 tr(eps)^2 + mu eps:eps),
and the rigid motions (translations, infinitesimal rotations) are its null
space.  The assembled operator inherits both; the split tiles the cube, and
the sizes match the paper's two matrices.
"""
import numpy as np
import pytest

import meshgen
from meshgen.elasticity import bsr_to_csr


def _lame(nu, E=1.0):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def _rigid_motions(coords):
    d = coords - coords.mean(axis=0)
    R = np.zeros((3 * len(coords), 6))
    R[0::3, 0] = R[1::3, 1] = R[2::3, 2] = 1.0
    R[1::3, 3], R[2::3, 3] = -d[:, 2], d[:, 1]
    R[0::3, 4], R[2::3, 4] = d[:, 2], -d[:, 0]
    R[0::3, 5], R[1::3, 5] = -d[:, 1], d[:, 0]
    return R


def test_element_energy_of_a_linear_field_is_exact():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((4, 3))
    nu = 0.3
    lam, mu = _lame(nu)
    K = meshgen.p1_element_stiffness(X, nu)
    G = rng.standard_normal((3, 3))
    u = (X @ G.T).ravel()                      # u(x_a) = G x_a, node-major
    eps = 0.5 * (G + G.T)
    V = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1))) / 6
    exact = V * (0.5 * lam * np.trace(eps) ** 2 + mu * np.sum(eps * eps))
    assert 0.5 * u @ K @ u == pytest.approx(exact, rel=1e-12)
    assert np.allclose(K, K.T, atol=1e-14 * abs(K).max())


def test_element_null_space_is_the_rigid_motions():
    X = np.array([[0.0, 0, 0], [1, 0.1, 0], [0.2, 1, 0.1], [0.1, 0.3, 1]])
    K = meshgen.p1_element_stiffness(X, 0.3)
    R = _rigid_motions(X)
    assert abs(K @ R).max() <= 1e-13 * abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert (abs(ev[:6]) <= 1e-12 * ev[-1]).all() and ev[6] > 1e-6 * ev[-1]


def test_assembled_operator_kernel_volume_and_load():
    rp, col, val, coords, fixed, tets, vol = meshgen.assemble_tets(6, clamp_x0=False)
    K = bsr_to_csr(rp, col, val)
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
    assert abs(K @ _rigid_motions(coords)).max() <= 1e-13 * abs(K).max()
    assert len(tets) == 6 * 5 ** 3 and len(tets) * vol == pytest.approx(1.0, rel=1e-14)
    # each cell's six tetrahedra have distinct vertex sets sharing the main diagonal
    cell = tets[::125][:6]
    assert len({tuple(sorted(t)) for t in cell}) == 6
    assert all(0 in t and 1 + 6 + 36 in t for t in cell)
    # consistent body force: int N_a dV sums to the volume
    p = meshgen.tet_cube(6)
    w = np.bincount(tets.ravel(), minlength=len(coords)) * vol / 4
    assert w.sum() == pytest.approx(1.0, rel=1e-14)
    assert np.allclose(p.b.reshape(-1, 3)[~p.fixed, 2], -w[~p.fixed])
    assert not p.b.reshape(-1, 3)[p.fixed].any()


def test_clamped_rows_are_identity_and_pattern_is_15_point():
    p = meshgen.tet_cube(7)
    A = p.csr()
    counts = np.diff(p.row_ptr)
    assert counts.max() == 15
    for r in np.flatnonzero(p.fixed)[:20]:
        assert p.col[p.row_ptr[r]:p.row_ptr[r + 1]].tolist() == [r]
        assert np.array_equal(p.val[p.row_ptr[r]], np.eye(3))
    for r in range(p.nb):
        c = p.col[p.row_ptr[r]:p.row_ptr[r + 1]]
        assert (np.diff(c) > 0).all() and r in c
    free = np.repeat(~p.fixed, 3)
    Af = A[free][:, free].toarray()
    assert np.linalg.eigvalsh(Af)[0] > 0


def test_sizes_match_the_paper_matrices():
    rod, hook = meshgen.rod_standin(), meshgen.hook_standin()
    assert rod.n == 81_000 and hook.n == 59_049
    # the paper's rod has 81,657 unknowns and 3,171,111 nonzeros, the hook
    # 59,718 and 2,309,832 (Section 4)
    assert abs(rod.csr().nnz / 3_171_111 - 1) < 0.02
    assert abs(hook.csr().nnz / 2_309_832 - 1) < 0.02
