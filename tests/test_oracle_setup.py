"""Pins for the oracle's SA-AMG setup (CPU only).

Each check is fixed by mathematics or by a hand-worked example, not by the
oracle's own code: graph invariants of the aggregation, aggregation results
traced by hand on small graphs, orthonormality and exact near-nullspace
reproduction of the tentative prolongation, exact reproduction of the rigid
body modes by the smoothed prolongation when every link is strong (A B = 0),
the 6x6 block structure of coarse matrices, and the smoother's defining
equations.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle
from oracle import setup as S


def _graph(N, edges, ratios=None):
    """StrengthGraph from an explicit (possibly asymmetric) list of directed links."""
    ratios = ratios or {}
    nbrs = [[] for _ in range(N)]
    for (i, j) in edges:
        nbrs[i].append(j)
    ptr = np.zeros(N + 1, dtype=np.int64)
    nbr, rat = [], []
    for i in range(N):
        for j in sorted(nbrs[i]):
            nbr.append(j)
            rat.append(ratios.get((i, j), ratios.get((j, i), 1.0)))
        ptr[i + 1] = len(nbr)
    rat = np.array(rat, dtype=np.float64)
    return S.StrengthGraph(N, ptr, np.array(nbr, dtype=np.int64), rat, np.sqrt(rat))


def _sym(edges):
    return edges + [(j, i) for (i, j) in edges]


# ---------------------------------------------------------------------------
# aggregation: hand-traced examples
# ---------------------------------------------------------------------------

def test_aggregation_chain_phase1_and_phase2():
    # path 0-1-...-8: seeds 0 -> {0,1}; 2 skipped (1 taken); 3 -> {2,3,4};
    # 5 skipped; 6 -> {5,6,7}; 8 skipped, then joins 7's aggregate in phase 2
    G = _graph(9, _sym([(i, i + 1) for i in range(8)]))
    agg, n = S.aggregate(G)
    assert n == 3
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2, 2, 2]


@pytest.mark.parametrize("r32,r35,expect", [
    (0.5, 0.9, 1),            # strictly stronger link to aggregate 1
    (0.9, 0.5, 0),            # strictly stronger link to aggregate 0
    (0.7, 0.7, 0),            # exact tie: lowest aggregate id
    (0.7 * (1 - 1e-13), 0.7, 0),  # within the 1e-12 slack: still a tie
    (0.7 * (1 - 1e-9), 0.7, 1),   # outside the slack: the stronger wins
])
def test_aggregation_phase2_strongest_and_ties(r32, r35, expect):
    # edges 0-1, 0-2, 2-3, 3-5, 4-5, 4-6: seeds 0 -> {0,1,2}, 4 -> {4,5,6};
    # node 3 (skipped in phase 1) joins the aggregate of its stronger link
    G = _graph(7, _sym([(0, 1), (0, 2), (2, 3), (3, 5), (4, 5), (4, 6)]),
               {(3, 2): r32, (3, 5): r35})
    agg, n = S.aggregate(G)
    assert n == 2
    assert agg[[0, 1, 2]].tolist() == [0, 0, 0] and agg[[4, 5, 6]].tolist() == [1, 1, 1]
    assert agg[3] == expect


def test_aggregation_isolated_nodes():
    G = _graph(5, _sym([(0, 1), (1, 2)]))
    agg, n = S.aggregate(G)
    # 0 seeds {0,1}; 2 is skipped (1 taken) and joins aggregate 0 in phase 2;
    # 3 and 4 have no strong neighbour
    assert agg.tolist() == [0, 0, 0, -1, -1] and n == 1


def test_aggregation_one_sided_link_never_pulls_in_isolated_node():
    # directed links 1 -> 0, 1 -> 2, 2 -> 1: node 0 has no strong neighbour of
    # its own, so it stays isolated although node 1 lists it
    G = _graph(3, [(1, 0), (2, 1), (1, 2)])
    agg, n = S.aggregate(G)
    assert agg.tolist() == [-1, 0, 0] and n == 1


def test_every_non_isolated_node_is_aggregated_after_phase2():
    rng = np.random.default_rng(7)
    for trial in range(20):
        N = 30
        edges = set()
        for _ in range(40):
            i, j = rng.integers(0, N, 2)
            if i != j:
                edges.add((int(i), int(j)))
                if rng.random() < 0.8:
                    edges.add((int(j), int(i)))
        G = _graph(N, sorted(edges), {e: float(rng.random()) for e in edges})
        agg, n = S.aggregate(G)
        iso = np.diff(G.ptr) == 0
        assert np.all(agg[~iso] >= 0) and np.all(agg[iso] == -1)


def test_aggregation_merges_rank_deficient_aggregate():
    # path 0-1-2-3-4 with non-collinear nodes: phase 1 gives {0,1} and {2,3,4};
    # two nodes only carry 5 independent rigid modes, so {0,1} merges into
    # its only neighbour aggregate and the survivors are renumbered.
    coords = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1], [0, 1, 1.0]])
    B = oracle.rigid_body_modes(coords)
    G = _graph(5, _sym([(0, 1), (1, 2), (2, 3), (3, 4)]))
    agg0, n0 = S.aggregate(G)
    assert agg0.tolist() == [0, 0, 1, 1, 1]
    agg, n = S.aggregate(G, B, 3)
    assert n == 1 and agg.tolist() == [0, 0, 0, 0, 0]


def _c1_level1(n=10, eps=0.08):
    p = meshgen.cube_c1(n)
    A = p.csr()
    G = S.strength_graph(A, 3, eps)
    B = oracle.rigid_body_modes(p.coords)
    return p, A, G, B


def test_strength_graph_symmetric_and_dirichlet_isolated():
    p, A, G, B = _c1_level1(6)
    links = set()
    for I in range(G.N):
        for J in G.neighbours(I)[0]:
            links.add((I, int(J)))
    assert all((J, I) in links for (I, J) in links)
    for I in np.flatnonzero(p.fixed):
        assert G.ptr[I + 1] == G.ptr[I]


def test_aggregation_invariants_cube():
    p, A, G, B = _c1_level1(10)
    agg, n = S.aggregate(G, B, 3)
    iso = np.diff(G.ptr) == 0
    # partition of the non-isolated nodes
    assert np.all(agg[iso] == -1) and np.all(agg[~iso] >= 0)
    assert set(agg[~iso].tolist()) == set(range(n))
    # each aggregate is connected in the strong graph and has full-rank modes
    for a in range(n):
        nodes = set(np.flatnonzero(agg == a).tolist())
        start = min(nodes)
        seen, stack = {start}, [start]
        while stack:
            I = stack.pop()
            for J in G.neighbours(I)[0].tolist():
                if J in nodes and J not in seen:
                    seen.add(J)
                    stack.append(J)
        assert seen == nodes
        rows = np.array(sorted(nodes))[:, None] * 3 + np.arange(3)
        assert np.linalg.matrix_rank(B[rows.ravel()]) == 6


# ---------------------------------------------------------------------------
# transfer operators
# ---------------------------------------------------------------------------

def test_tentative_prolongation_orthonormal_and_exact_on_modes():
    p, A, G, B = _c1_level1(8)
    agg, n = S.aggregate(G, B, 3)
    Pt, Bc = S.tentative_prolongation(agg, n, B, 3)
    PtP = (Pt.T @ Pt).toarray()
    assert np.abs(PtP - np.eye(6 * n)).max() < 1e-13
    rows = np.repeat(agg >= 0, 3)
    assert np.abs((Pt @ Bc)[rows] - B[rows]).max() < 1e-13 * np.abs(B).max()
    assert abs(Pt[~rows]).max() == 0.0 if (~rows).any() else True
    # R factors: upper triangular, positive diagonal
    for a in range(n):
        R = Bc[6 * a:6 * a + 6]
        assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) > 0)


def test_tentative_matches_library_qr_after_sign_normalisation():
    rng = np.random.default_rng(1)
    Ba = rng.standard_normal((27, 6))
    Q, R = S.local_qr(Ba)
    Q2, R2 = np.linalg.qr(Ba)
    s = np.sign(np.diag(R2))
    assert np.allclose(Q, Q2 * s, atol=1e-14) and np.allclose(R, R2 * s[:, None], atol=1e-13)
    assert np.allclose(Q @ R, Ba, atol=1e-13)


def _free_cube(n):
    h = 1.0 / n
    rp, col, val, coords, fixed = meshgen.assemble_box(n, n, n, h, h, h, 0.3, clamp_x0=False)
    return meshgen.bsr_to_csr(rp, col, val), coords


def test_smoothed_prolongation_reproduces_modes_when_all_links_strong():
    """Free mesh, eps = 0: A_F = A and A B = 0, so P B_c = B and A_c B_c = 0,
    on two consecutive levels."""
    A, coords = _free_cube(6)
    B = oracle.rigid_body_modes(coords)
    b = 3
    scale = abs(A).max()
    for level in range(2):
        G = S.strength_graph(A, b, 0.0)
        agg, n = S.aggregate(G, B, b)
        Pt, Bc = S.tentative_prolongation(agg, n, B, b)
        P = S.smoothed_prolongation(A, G, b, Pt, 2.0 / 3.0)
        assert np.abs(P @ Bc - B).max() < 1e-11 * np.abs(B).max()
        Ac = (P.T @ A @ P).tocsr()
        scale *= abs(P).max() ** 2
        assert np.abs(Ac @ Bc).max() < 1e-12 * scale * np.abs(Bc).max() * A.shape[0]
        A, B, b = Ac, Bc, 6
    assert n >= 1


def test_filtered_matrix_lumping_preserves_row_sums():
    p, A, G, B = _c1_level1(6)
    AF = S.filtered_matrix(A, G, 3)
    one = np.ones(A.shape[0])
    assert np.abs(AF @ one - A @ one).max() < 1e-13 * abs(A).max()
    # strong blocks and diagonal blocks are untouched off the scalar diagonal
    D = (AF - A).tocoo()
    off = D.row != D.col
    nz = np.abs(D.data[off]) > 0
    # every changed off-diagonal entry was removed (weak block), never altered
    rows, cols = D.row[off][nz], D.col[off][nz]
    assert np.all(np.asarray(AF[rows, cols]).ravel() == 0)


def test_coarse_matrix_has_6x6_block_structure_and_is_spd():
    p = meshgen.cube_c1(8)
    h = oracle.build_hierarchy(p.csr(), p.coords, oracle.AmgParams(coarse_enough=200))
    assert len(h.levels) >= 2
    for lev in h.levels[1:]:
        Ac = lev.A.tocsr()
        N = lev.n // 6
        # every scalar row of coarse node I touches the same set of coarse nodes
        for I in range(N):
            sets = [frozenset((Ac.indices[Ac.indptr[i]:Ac.indptr[i + 1]] // 6).tolist())
                    for i in range(6 * I, 6 * I + 6)]
            assert len(set(sets)) == 1
        # and a present 6x6 block is dense (up to exact cancellations)
        Ad = lev.A.toarray().reshape(N, 6, N, 6)
        nz = (Ad != 0).sum(axis=(1, 3))
        assert np.all((nz == 0) | (nz >= 34))
        assert abs(lev.A - lev.A.T).max() <= 1e-13 * abs(lev.A).max()
        assert np.linalg.eigvalsh(lev.A.toarray()).min() > 0


def test_jacobi_smoother_definition_and_damping_bound():
    p = meshgen.cube_lognormal(5, seed=3)
    A = p.csr()
    M, Mt = S.jacobi_smoother(A)
    Ad, Md = A.toarray(), M.toarray()
    lam_d = np.linalg.eigvals(np.linalg.solve(S._diag_blocks(A)[0], np.eye(3)))  # smoke
    omega = None
    for I in range(A.shape[0] // 3):
        prod = Md[3 * I:3 * I + 3, 3 * I:3 * I + 3] @ Ad[3 * I:3 * I + 3, 3 * I:3 * I + 3]
        if omega is None:
            omega = prod[0, 0]
        assert np.allclose(prod, omega * np.eye(3), atol=1e-13)
    # omega * lambda_max(D^-1 A) < 2: the damped sweep is an A-norm contraction
    lam = np.linalg.eigvals(Md @ Ad).real.max()
    assert lam < 2.0
    assert np.linalg.eigvalsh(Md + Md.T - Md.T @ Ad @ Md).min() > 0
    assert np.isfinite(lam_d).all()


def test_spai0_blocks_are_the_frobenius_minimiser():
    # each undamped block row solves min ||E_I - M_I A_{I,:}||_F, a least
    # squares problem in M_I^T that numpy's lstsq solves independently
    p = meshgen.cube_lognormal(4, seed=5)
    A = p.csr()
    M, Mt = S.spai0_smoother(A, omega=1.0)
    Ad, Md = A.toarray(), M.toarray()
    n = Ad.shape[0]
    for I in range(n // 3):
        rows = slice(3 * I, 3 * I + 3)
        E = np.eye(n)[rows]
        sol, *_ = np.linalg.lstsq(Ad[rows].T, E.T, rcond=None)
        assert np.allclose(Md[rows, rows], sol.T, rtol=1e-10, atol=1e-12), I
    assert abs(Mt - M.T).max() == 0.0
    # and no block-diagonal perturbation lowers the Frobenius residual
    rng = np.random.default_rng(0)
    base = np.linalg.norm(np.eye(n) - Md @ Ad)
    for _ in range(3):
        dM = S._block_diag_matrix(1e-3 * rng.standard_normal((n // 3, 3, 3))).toarray()
        assert np.linalg.norm(np.eye(n) - (Md + dM) @ Ad) > base


def test_spai0_of_block_diagonal_matrix_is_its_inverse():
    rng = np.random.default_rng(1)
    blocks = rng.standard_normal((7, 3, 3))
    blocks = blocks @ np.transpose(blocks, (0, 2, 1)) + 3 * np.eye(3)
    A = S._block_diag_matrix(blocks)
    M, _ = S.spai0_smoother(A, omega=1.0)
    assert np.allclose(M.toarray(), np.linalg.inv(A.toarray()), rtol=1e-12, atol=1e-14)


def test_spai0_damping_gives_a_contraction_and_a_symmetric_vcycle():
    p = meshgen.cube_lognormal(5, seed=3)
    A = p.csr()
    Ad = A.toarray()
    M0, _ = S.spai0_smoother(A, omega=1.0)
    # undamped SPAI-0 diverges on these matrices: lambda_max(M_0 A) > 2
    assert np.abs(np.linalg.eigvals(M0.toarray() @ Ad)).max() > 2.0
    M, Mt = S.spai0_smoother(A)
    Md = M.toarray()
    Sm = np.eye(Ad.shape[0]) - Md @ Ad
    # the damped sweep contracts the energy norm: A - S^T A S > 0
    assert np.linalg.eigvalsh(Ad - Sm.T @ Ad @ Sm).min() > 0
    h = oracle.build_hierarchy(A, p.coords, oracle.AmgParams(smoother="spai0", coarse_enough=100))
    assert len(h.levels) >= 2
    n = A.shape[0]
    B = np.column_stack([oracle.vcycle(h, np.eye(n)[:, j]) for j in range(n)])
    assert np.allclose(B, B.T, rtol=0, atol=1e-10 * np.abs(B).max())
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    r = oracle.amg_pcg(h, p.b, tol=1e-8)
    assert r.converged and oracle.true_residual_norm(A, p.b, r.x) <= 1e-8


def test_hierarchy_levels_and_stop_rule():
    p = meshgen.cube_c1(10)
    h = oracle.build_hierarchy(p.csr(), p.coords)
    sizes = h.sizes()
    assert sizes[0] == 3993 and sizes[-1] <= 3000
    assert all(s % 6 == 0 for s in sizes[1:])
    assert all(sizes[i + 1] <= 0.9 * sizes[i] for i in range(len(sizes) - 1))
