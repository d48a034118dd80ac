"""Pins for the oracle's V-cycle and PCG (CPU only).

* the V-cycle, applied to unit vectors, equals the recursive closed form
  B_l = (I - E_l) A_l^{-1}, E_l = (I - M_l^T A_l)(I - P_l B_{l+1} R_l A_l)(I - M_l A_l),
  B_L = A_L^{-1} (one pre- and one post-sweep), and is symmetric positive
  definite, as CG requires;
* CG iterates equal scipy's cg with the same preconditioner;
* converged solutions equal a dense direct solve on small meshes;
* the block form (scipy BSR with 3x3 blocks) of every level applies the same
  V-cycle as the scalar form (the paper's block and scalar solvers share
  iteration counts, Tables 1 and 2);
* the rigid body modes cut the iteration count (Section 4, Tables 1 and 2:
  about 3x fewer iterations with the near-nullspace).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import meshgen
import oracle
from oracle import setup as S
from oracle.solve import vcycle, pcg, amg_pcg


def _small_hierarchy(n=6, coarse=100, **kw):
    p = meshgen.cube_lognormal(n, seed=4)
    h = oracle.build_hierarchy(p.csr(), p.coords, oracle.AmgParams(coarse_enough=coarse, **kw))
    return p, h


def _closed_form(h, l=0):
    lev = h.levels[l]
    A = lev.A.toarray()
    if lev.is_coarsest:
        return np.linalg.inv(A)
    I = np.eye(lev.n)
    M, Mt = lev.M.toarray(), lev.Mt.toarray()
    P, R = lev.P.toarray(), lev.R.toarray()
    Bc = _closed_form(h, l + 1)
    E = (I - Mt @ A) @ (I - P @ Bc @ R @ A) @ (I - M @ A)
    return (I - E) @ np.linalg.inv(A)


def test_vcycle_equals_closed_form_and_is_spd():
    p, h = _small_hierarchy(6, coarse=60)
    assert len(h.levels) >= 3
    n = h.levels[0].n
    V = np.column_stack([vcycle(h, e) for e in np.eye(n)])
    Bref = _closed_form(h)
    assert np.abs(V - Bref).max() <= 1e-9 * np.abs(Bref).max()
    assert np.abs(V - V.T).max() <= 1e-12 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0


def test_pcg_iterates_match_scipy_cg():
    p, h = _small_hierarchy(6)
    A = h.levels[0].A
    Mop = spla.LinearOperator(A.shape, matvec=lambda r: vcycle(h, r))
    for k in (1, 3, 7):
        ours = pcg(A, p.b, lambda r: vcycle(h, r), tol=1e-30, maxiter=k)
        ref, info = spla.cg(A, p.b, rtol=1e-30, atol=0.0, maxiter=k, M=Mop)
        assert ours.iters == k
        assert np.linalg.norm(ours.x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_identity_preconditioned_cg_finishes_in_n_steps():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    A = sp.csr_matrix(Q @ np.diag(np.linspace(1, 4, 8)) @ Q.T)
    b = rng.standard_normal(8)
    res = pcg(A, b, tol=1e-12)
    assert res.converged and res.iters <= 8
    assert np.allclose(res.x, np.linalg.solve(A.toarray(), b), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("n", [4, 10])
def test_amg_pcg_solution_matches_dense_solve(n):
    p = meshgen.cube_c1(n)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords)
    res = amg_pcg(h, p.b, tol=1e-10)
    x = sla.solve(A.toarray(), p.b, assume_a="pos")
    assert res.converged and res.rel_true_residual <= 1e-10
    assert np.linalg.norm(res.x - x) <= 1e-7 * np.linalg.norm(x)


def test_c1_converges_to_1e8():
    p = meshgen.cube_c1(10)
    A = p.csr()
    h = oracle.build_hierarchy(A, p.coords)
    res = amg_pcg(h, p.b, tol=1e-8)
    assert res.converged
    assert oracle.true_residual_norm(A, p.b, res.x) <= 1e-8
    assert 5 <= res.iters <= 40


def test_block_form_vcycle_equals_scalar_form():
    p, h = _small_hierarchy(8, coarse=200)
    hb = oracle.Hierarchy([S.Level(A=lev.A, b=lev.b) for lev in h.levels], h.params)
    for lb, lev in zip(hb.levels, h.levels):
        conv = lambda X: None if X is None else sp.bsr_matrix(X, blocksize=(3, 3))  # noqa: E731
        lb.A = conv(lev.A)
        lb.P, lb.R, lb.M, lb.Mt = conv(lev.P), conv(lev.R), conv(lev.M), conv(lev.Mt)
        lb.chol = lev.chol
    rng = np.random.default_rng(9)
    r = rng.standard_normal(h.levels[0].n)
    a, b = vcycle(h, r), vcycle(hb, r)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


def test_rigid_body_modes_reduce_iterations():
    # cube 16^3 with two levels: 21 iterations with the modes, 43 without
    p = meshgen.cube_c1(16)
    A = p.csr()
    prm = dict(coarse_enough=500)
    with_ns = amg_pcg(oracle.build_hierarchy(A, p.coords, oracle.AmgParams(**prm)), p.b)
    without = amg_pcg(oracle.build_hierarchy(
        A, p.coords, oracle.AmgParams(use_nullspace=False, **prm)), p.b)
    assert with_ns.converged and without.converged
    assert 2 * with_ns.iters <= without.iters + 2


def test_zero_rhs_and_breakdown():
    p, h = _small_hierarchy(4)
    A = h.levels[0].A
    res = pcg(A, np.zeros(A.shape[0]), lambda r: vcycle(h, r))
    assert res.iters == 0 and res.converged and not res.x.any()
    neg = pcg(-A, p.b, lambda r: vcycle(h, r))
    assert neg.breakdown and not neg.converged
