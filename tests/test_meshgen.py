"""Pins for the synthetic elasticity inputs (CPU only).

Closed forms that the inputs must satisfy whatever the solver does:
rigid motions have zero strain energy, a linear displacement field has the
exact strain energy of a homogeneous strain, loads integrate to the applied
totals, and the block counts of the 10^3 cube match its 27-point stencil.
"""
import numpy as np
import pytest

import meshgen
import oracle


def _free_box(nx, ny, nz, hx, hy, hz, nu, E=None):
    rp, col, val, coords, fixed = meshgen.assemble_box(nx, ny, nz, hx, hy, hz, nu, E,
                                                       clamp_x0=False)
    A = meshgen.bsr_to_csr(rp, col, val)
    return A, coords


def test_element_stiffness_kernel_is_rigid_motions():
    K = meshgen.q1_element_stiffness(0.3, 0.2, 0.5, 0.3)
    assert np.allclose(K, K.T, atol=0)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == 6
    assert ev[6] > 1e-4 * ev.max()


def test_rigid_body_modes_in_kernel_of_free_stiffness():
    rng = np.random.default_rng(11)
    E = np.exp(rng.standard_normal(3 * 4 * 2))
    A, coords = _free_box(3, 4, 2, 0.25, 0.4, 0.3, 0.3, E)
    B = oracle.rigid_body_modes(coords)
    KB = A @ B
    scale = abs(A).max() * np.abs(B).max()
    assert np.abs(KB).max() <= 1e-12 * scale * A.shape[0] ** 0.5
    # and B has full rank 6
    assert np.linalg.matrix_rank(B) == 6


@pytest.mark.parametrize("nu", [0.3, 0.45])
def test_patch_test_strain_energy(nu):
    """u = eps x gives 1/2 u^T K u = 1/2 V (lambda tr(eps)^2 + 2 mu eps:eps)."""
    nx, ny, nz, hx, hy, hz = 3, 2, 4, 0.5, 0.25, 0.2
    A, coords = _free_box(nx, ny, nz, hx, hy, hz, nu)
    rng = np.random.default_rng(5)
    G = rng.standard_normal((3, 3))
    eps = 0.5 * (G + G.T)
    u = (coords @ eps.T).ravel()
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    V = nx * hx * ny * hy * nz * hz
    exact = 0.5 * V * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    got = 0.5 * u @ (A @ u)
    assert abs(got - exact) <= 1e-12 * abs(exact)


def test_cube10_counts_and_dirichlet_rows():
    p = meshgen.cube_c1(10)
    assert p.nb == 1331 and p.n == 3993 and p.nnzb == 27029
    rp, col = p.row_ptr, p.col
    assert rp.dtype == np.int32 and col.dtype == np.int32
    for I in np.flatnonzero(p.fixed):
        assert rp[I + 1] - rp[I] == 1 and col[rp[I]] == I
        assert np.array_equal(p.val[rp[I]], np.eye(3))
        assert np.all(p.b[3 * I:3 * I + 3] == 0)
    # columns sorted, diagonal present in every row
    for I in range(p.nb):
        c = col[rp[I]:rp[I + 1]]
        assert np.all(np.diff(c) > 0) and I in c
    A = p.csr()
    assert abs(A - A.T).max() == 0.0


def test_load_totals():
    # body force on a free cube integrates to -volume in z
    rp, col, val, coords, fixed = meshgen.assemble_box(4, 4, 4, 0.25, 0.25, 0.25, 0.3,
                                                       clamp_x0=False)
    from meshgen.elasticity import _body_force, _tip_load
    b = _body_force(4, 4, 4, 0.25, 0.25, 0.25, fixed).reshape(-1, 3)
    assert np.allclose(b.sum(axis=0), [0, 0, -1.0], atol=1e-14)
    t = _tip_load(8, 2, 2, 0.5, 0.5, 0.5, fixed=np.zeros(9 * 3 * 3, dtype=bool)).reshape(-1, 3)
    assert np.allclose(t.sum(axis=0), [0, 0, -1.0], atol=1e-14)


def test_seeded_workloads_are_reproducible():
    a = meshgen.cube_lognormal(4, seed=0)
    b = meshgen.cube_lognormal(4, seed=0)
    assert np.array_equal(a.val, b.val)
    c = meshgen.cube_inclusions(12, n_incl=5, radius_elems=2)
    assert c.val.max() > 100  # stiff inclusions present
    m = meshgen.cube_multi_rhs(4, 3)
    assert m.b.shape == (3 * 125, 3) and np.all(m.b[np.repeat(m.fixed, 3)] == 0)
    edges = [pp.dims[0] for pp in meshgen.batch_cubes(6, 2, 4)]
    assert all(2 <= e <= 4 for e in edges)
