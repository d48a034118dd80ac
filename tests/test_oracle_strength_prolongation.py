"""Hand-worked pins for the strength graph and the smoothed prolongation
(Algorithm 1: strong couplings decide the aggregates, the tentative
prolongation is smoothed by one damped Jacobi step on the filtered matrix).

Every expected value below was worked out by hand from the readings
(strength: s_IJ = Frobenius norm of node block A_IJ, J strong for I iff
s_IJ^2 >= eps_l^2 s_II s_JJ, eps_l = 0.08 * 0.5^(l-1); prolongation:
P = (I - omega D^{-1} A_F) P^ with omega = 2/3, D the scalar diagonal of A,
A_F = A without the weak node blocks, whose entries are added to the scalar
diagonal of their rows).  The examples are chosen so that each plausible
slip gives a different answer: comparing the ratio with eps instead of
eps^2, using sqrt(s_II s_JJ), a max-entry instead of the Frobenius block
norm, no halving of eps on level 2; omega = 4/3, D = diag(A_F), a block
diagonal D, keeping the weak block, or not lumping it.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle
from oracle import setup as S


def _assemble(nodes, blocks):
    """Symmetric scalar matrix from upper node blocks {(I, J): 3x3}."""
    A = np.zeros((3 * nodes, 3 * nodes))
    for (I, J), blk in blocks.items():
        blk = np.asarray(blk, dtype=np.float64)
        A[3 * I:3 * I + 3, 3 * J:3 * J + 3] = blk
        if I != J:
            A[3 * J:3 * J + 3, 3 * I:3 * I + 3] = blk.T
    return sp.csr_matrix(A)


def _strength_example():
    # diagonal blocks with Frobenius norms s = (3, 6, 3, 12)
    D0 = np.diag([2.0, 2.0, 1.0])      # sqrt(4+4+1) = 3
    D1 = np.diag([4.0, 4.0, 2.0])      # sqrt(16+16+4) = 6
    D2 = np.diag([1.0, 2.0, 2.0])      # sqrt(1+4+4) = 3
    D3 = np.diag([8.0, 8.0, 4.0])      # sqrt(64+64+16) = 12
    z = np.zeros((3, 3))

    def blk(entries):
        b = z.copy()
        for (i, j), v in entries.items():
            b[i, j] = v
        return b

    blocks = {
        (0, 0): D0, (1, 1): D1, (2, 2): D2, (3, 3): D3,
        # s01^2 = 0.09 + 0.09 = 0.18, s00 s11 = 18: ratio 0.01
        (0, 1): blk({(0, 0): 0.3, (1, 2): -0.3}),
        # s13^2 = 0.36 (one entry 0.6), s11 s33 = 72: ratio 0.005
        (1, 3): blk({(2, 1): 0.6}),
        # s02^2 = 0.027 (0.15^2 + 0.06^2 + 0.03^2 = 0.0225 + 0.0036 + 0.0009), s00 s22 = 9: ratio 0.003
        (0, 2): blk({(0, 0): 0.15, (1, 1): 0.06, (2, 0): -0.03}),
        # s23^2 = 0.2304 (one entry 0.48), s22 s33 = 36: ratio 0.0064, exactly eps^2 at 0.08
        (2, 3): blk({(1, 0): 0.48}),
        # s03^2 = 0.225 (0.45^2 + 0.15^2 = 0.2025 + 0.0225), s00 s33 = 36: ratio 0.00625, just below 0.0064
        (0, 3): blk({(0, 2): 0.45, (1, 1): -0.15}),
        # s12^2 = 0.018 (0.09^2 + 0.09^2 + 0.0018), s11 s22 = 18: ratio 0.001
        (1, 2): blk({(0, 1): 0.09, (1, 0): -0.09, (2, 2): 0.03 * np.sqrt(2.0)}),
    }
    return _assemble(4, blocks)


def _links(G):
    out = {}
    for I in range(G.N):
        nb, ratio, norm = G.neighbours(I)
        for J, r, s in zip(nb.tolist(), ratio.tolist(), norm.tolist()):
            out[(I, J)] = (r, s)
    return out


def test_strength_example_block_norms_are_as_worked():
    A = _strength_example().toarray()
    fro = lambda I, J: np.linalg.norm(A[3 * I:3 * I + 3, 3 * J:3 * J + 3])
    assert [fro(I, I) for I in range(4)] == pytest.approx([3, 6, 3, 12], rel=1e-15)
    sq = {(0, 1): 0.18, (1, 3): 0.36, (0, 2): 0.027, (2, 3): 0.2304, (0, 3): 0.225, (1, 2): 0.018}
    for (I, J), v in sq.items():
        assert fro(I, J) ** 2 == pytest.approx(v, rel=1e-13)


@pytest.mark.parametrize("eps,strong", [
    # level 1 (eps^2 = 0.0064): ratio 0.01 strong, 0.0064 strong (tie), 0.00625, 0.005, 0.003, 0.001 weak
    (0.08, {(0, 1), (2, 3)}),
    # level 2 (eps^2 = 0.0016): 0.00625, 0.005 and 0.003 become strong, 0.001 stays weak
    (0.04, {(0, 1), (2, 3), (0, 3), (1, 3), (0, 2)}),
    # level 3 (eps^2 = 0.0004): every link
    (0.02, {(0, 1), (2, 3), (0, 3), (1, 3), (0, 2), (1, 2)}),
])
def test_strength_graph_hand_worked(eps, strong):
    G = S.strength_graph(_strength_example(), 3, eps)
    links = _links(G)
    expect = strong | {(j, i) for (i, j) in strong}
    assert set(links) == expect
    ratios = {(0, 1): 0.01, (2, 3): 0.0064, (0, 3): 0.00625, (1, 3): 0.005, (0, 2): 0.003, (1, 2): 0.001}
    for (i, j), (r, s) in links.items():
        key = (min(i, j), max(i, j))
        assert r == pytest.approx(ratios[key], rel=1e-12)
        assert s * s == pytest.approx(ratios[key] * {0: 3, 1: 6, 2: 3, 3: 12}[i] * {0: 3, 1: 6, 2: 3, 3: 12}[j],
                                      rel=1e-12)


def test_strength_threshold_decays_by_half_per_level():
    """The level thresholds of a four-level hierarchy are 0.08, 0.04, 0.02,
    0.01 (reading: halved per level), and the level-2 aggregates are those of
    the strength graph at 0.04, not at 0.08 (the test is sensitive to it)."""
    p = meshgen.cube_c1(10)
    h = oracle.build_hierarchy(p.csr(), p.coords, oracle.AmgParams(coarse_enough=60))
    assert len(h.levels) >= 3
    assert [lev.eps for lev in h.levels[:4]] == pytest.approx([0.08, 0.04, 0.02, 0.01][:len(h.levels[:4])],
                                                               rel=1e-15)
    lev2 = h.levels[1]
    agg04, n04 = S.aggregate(S.strength_graph(lev2.A, 6, 0.04), lev2.B, 6)
    agg08, n08 = S.aggregate(S.strength_graph(lev2.A, 6, 0.08), lev2.B, 6)
    assert np.array_equal(lev2.agg, agg04) and lev2.n_agg == n04
    assert not (n08 == n04 and np.array_equal(agg04, agg08))


def _prolongation_example():
    """Three nodes; node blocks 0-1 and 1-2 strong, 0-2 weak (ratios 0.049,
    0.133 and 0.00044 against eps^2 = 0.0064)."""
    blocks = {
        (0, 0): [[4.0, 1.0, 0.0], [1.0, 4.0, 0.0], [0.0, 0.0, 4.0]],
        (1, 1): np.eye(3) * 5.0,
        (2, 2): np.eye(3) * 6.0,
        (0, 1): -np.eye(3),
        (1, 2): -2.0 * np.eye(3),
        (0, 2): [[-0.1, 0.05, 0.0], [0.0, -0.1, 0.0], [0.0, 0.0, -0.1]],
    }
    return _assemble(3, blocks)


def test_prolongation_example_strength():
    G = S.strength_graph(_prolongation_example(), 3, 0.08)
    assert set(_links(G)) == {(0, 1), (1, 0), (1, 2), (2, 1)}


def test_filtered_matrix_hand_worked():
    A = _prolongation_example()
    G = S.strength_graph(A, 3, 0.08)
    AF = S.filtered_matrix(A, G, 3).toarray()
    # weak block 0-2 removed, its row sums lumped into the scalar diagonal:
    # rows 0..2 get -0.05, -0.1, -0.1; rows 6..8 (its transpose) -0.1, -0.05, -0.1
    assert np.diag(AF).tolist() == pytest.approx([3.95, 3.9, 3.9, 5, 5, 5, 5.9, 5.95, 5.9], abs=1e-15)
    assert np.all(AF[0:3, 6:9] == 0) and np.all(AF[6:9, 0:3] == 0)
    assert AF[0, 1] == 1.0 and AF[0, 3] == -1.0 and AF[3, 6] == -2.0


def test_smoothed_prolongation_hand_worked():
    """P = (I - 2/3 D^{-1} A_F) P^ for P^ = [e_0 + e_3, e_8] (aggregate {0, 1}
    carrying the x mode, aggregate {2} the z mode), D = diag(A) = (4,4,4,5,5,5,6,6,6).
    A_F P^ column 0 = (2.95, 1, 0, 4, 0, 0, -2, 0, 0), column 1 = (0, 0, 0, 0, 0, -2, 0, 0, 5.9)."""
    A = _prolongation_example()
    G = S.strength_graph(A, 3, 0.08)
    Pt = sp.csr_matrix(([1.0, 1.0, 1.0], ([0, 3, 8], [0, 0, 1])), shape=(9, 2))
    P = S.smoothed_prolongation(A, G, 3, Pt, 2.0 / 3.0).toarray()
    expect = np.zeros((9, 2))
    expect[:, 0] = [1 - 2.95 / 6, -1 / 6, 0, 7 / 15, 0, 0, 2 / 9, 0, 0]
    expect[:, 1] = [0, 0, 0, 0, 0, 4 / 15, 0, 0, 1 - 5.9 / 9]
    assert np.abs(P - expect).max() < 1e-14
    # the slips this example separates give other first entries:
    # omega 4/3 -> 1 - 2.95/3; D = diag(A_F) -> 1 - (2/3)(2.95/3.95); no lumping -> 1 - (2/3)(3/4)
    for wrong in (1 - 2.95 / 3, 1 - (2 / 3) * (2.95 / 3.95), 1 - (2 / 3) * (3 / 4)):
        assert abs(P[0, 0] - wrong) > 1e-3
    # keeping the weak block would give P[6, 0] = (2/3)(2.1/6), a block D^{-1} would move P[1, 0]
    assert abs(P[6, 0] - (2 / 3) * (2.1 / 6)) > 1e-3
    Dblk = np.array([[4.0, 1.0, 0.0], [1.0, 4.0, 0.0], [0.0, 0.0, 4.0]])
    assert abs(P[1, 0] - (-(2 / 3) * np.linalg.solve(Dblk, [2.95, 1.0, 0.0])[1])) > 1e-3


def test_build_hierarchy_uses_omega_two_thirds():
    """The hierarchy's P on level 1 is the hand-worked formula with omega = 2/3
    applied to its own P^ (and not 4/3)."""
    p = meshgen.cube_c1(6)
    h = oracle.build_hierarchy(p.csr(), p.coords, oracle.AmgParams(coarse_enough=200))
    lev = h.levels[0]
    assert lev.Ptent is not None
    A = lev.A
    G = S.strength_graph(A, 3, 0.08)
    AFPt = (S.filtered_matrix(A, G, 3) @ lev.Ptent).toarray()
    D = A.diagonal()
    P = lev.P.toarray()
    Pt = lev.Ptent.toarray()
    # omega recovered entry by entry where the correction is not negligible
    corr = AFPt / D[:, None]
    mask = np.abs(corr) > 1e-3
    omega = (Pt[mask] - P[mask]) / corr[mask]
    assert np.abs(omega - 2.0 / 3.0).max() < 1e-10
