"""Smoothed-aggregation AMG setup in scalar CSR (oracle; test infrastructure only).

Follows the setup loop of Algorithm 1 of the paper (Section 2): starting from
A_1 = A and B_1 = B (the rigid body modes), while A_i is too large for a direct
solve, build P_i and B_{i+1} from A_i and B_i, set R_i = P_i^T, build the
smoother S_i from A_i, and form the Galerkin product A_{i+1} = R_i A_i P_i;
finally factor the coarsest A_L for a direct solve.  Everything here is done
in scalar arithmetic, which is how the paper's "NS Scalar" solver (Section 4)
and the scalar coarsening under its "as_scalar" wrapper (Section 3) work.

The paper only names the ingredients (aggregation, tentative prolongation
from the near-nullspace, smoothing of the prolongation) without formulas, and
its experiments use ILU(0), which is here beside the block-Jacobi / SPAI-0
smoothers of the GPU path.  The readings used (each also listed in the design
notes):

* node size b = 3 on level 1 (one mesh node), 6 on coarser levels (one
  aggregate carries 6 near-nullspace coefficients);
* strength: s_IJ = Frobenius norm of the b x b node block A_IJ; J != I is a
  strong neighbour of I iff s_IJ^2 >= eps_l^2 s_II s_JJ (1 - 1e-12), with
  eps_l = eps_strong * eps_decay^(l-1) (0.08, halved per level);
* aggregation: greedy, nodes in increasing order --
  (1) I with no strong neighbour is isolated (never aggregated, zero rows in P);
      otherwise, if I and all its strong neighbours are unaggregated, I and
      its non-isolated strong neighbours form a new aggregate;
  (2) each remaining non-isolated node joins the phase-1 aggregate of its
      strongest strong neighbour (snapshot after phase 1), the ratio
      s_IJ^2/(s_II s_JJ) compared with 1e-12 relative slack, ties to the
      lowest aggregate id.  After this phase every non-isolated node is
      aggregated: a node left out by phase 1 was skipped because one of its
      strong neighbours was already taken, and that neighbour is a candidate
      here, so a third "leftover" phase would never run;
  (3) an aggregate whose local near-nullspace block is rank deficient
      (fewer than 6 rows, or min|R_kk| / max|R_kk| < 1e-10 in its thin QR) is
      merged into the neighbouring aggregate with the largest sum of s_IJ over
      the strong links between them (ties: lowest id, 1e-12 slack); passes over
      the aggregates in increasing id repeat until none merges; the surviving
      aggregates are then renumbered in increasing old id;
* tentative prolongation: per aggregate a, rows ordered by node id then
  component, B_a = Q_a R_a (thin QR with diag(R_a) > 0, unique for full rank),
  P^[rows(a), 6a:6a+6] = Q_a and B_{i+1}[6a:6a+6] = R_a;
* filtering and smoothing: A_F keeps the diagonal and the strong node blocks,
  every scalar entry of a weak block is added to the scalar diagonal of its row;
  P = (I - omega_p D^{-1} A_F) P^ with omega_p = 2/3 and D the scalar diagonal
  of A itself (the lumped diagonal of A_F can turn negative for elasticity
  blocks, so it is not used for the scaling);
* smoother (the paper's runs use ILU(0); the Jacobi-type smoothers it names
  as SpMV-dominated are used here): damped block Jacobi M_I = omega_j (A_II)^{-1} on the 3x3 diagonal
  blocks with omega_j = 4 / (3 lambda^), lambda^ = 30 power steps on
  D^{-1} A_l from x_i = (-1)^i (a fixed 2/3 lets omega_j lambda_max exceed 2 on
  stiff or heterogeneous meshes, which breaks the positive definiteness CG
  needs).  Block SPAI-0 (the block-diagonal minimiser of ||I - M A||_F,
  M_I = A_II (sum_J A_IJ A_IJ^T)^{-1}) is the second smoother; undamped it
  gives lambda_max(M A) > 2 on these elasticity matrices (a divergent sweep),
  so it takes the same damping 4 / (3 lambda^) with lambda^ from the power
  steps on M A; its blocks are not symmetric, so the post-sweep applies M^T
  and the V-cycle stays symmetric.  Block ILU(0) (the paper's smoother) is
  undamped: x <- x + (L U)^{-1} (f - A x) with L, U the incomplete factors on
  A's own 3x3 block pattern, the same operator before and after the coarse
  correction (L U is symmetric for symmetric A);
* stopping: a level with n_l <= coarse_enough (3000 unknowns) or the
  max_levels-th level is the coarsest; if an aggregation step would leave more
  than 0.9 n_l unknowns (or none), the current level becomes the coarsest;
* coarsest: dense Cholesky factorisation of A_L.

Parity pins (tests): K B = 0 on free meshes; P^T P^ = I and P^ B_{i+1} = B_i;
P B_{i+1} = B_i and A_{i+1} B_{i+1} = 0 on free meshes where every link is
strong; hand-worked aggregation examples; the 6x6 block pattern of coarse
levels; smoother optimality conditions; the V-cycle closed form; ILU(0)
equal to the exact block LU without fill, (L U)_ij = A_ij on the pattern,
U = D L^T, and its relaxation contracting.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .nullspace import rigid_body_modes

TIE_SLACK = 1e-12
RANK_TOL = 1e-10


@dataclasses.dataclass
class AmgParams:
    eps_strong: float = 0.08
    eps_decay: float = 0.5
    omega_p: float = 2.0 / 3.0
    smoother: str = "jacobi"        # "jacobi", "spai0" (damped block), "ilu0", "ilu0_mc" (multicolour order)
    omega_j: Optional[float] = None  # None: 4 / (3 lambda_max(M_0 A)) per level (M_0 undamped)
    npre: int = 1
    npost: int = 1
    coarse_enough: int = 3000
    max_levels: int = 10
    use_nullspace: bool = True      # False: constant vectors per dof (no rigid rotations)
    smoother_levels: Optional[int] = None  # "ilu0"/"ilu0_mc" on the first k levels only, block Jacobi below


@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    b: int                                   # node size (3 or 6)
    eps: float = 0.0
    P: Optional[sp.csr_matrix] = None
    R: Optional[sp.csr_matrix] = None
    Ptent: Optional[sp.csr_matrix] = None
    M: Optional[sp.csr_matrix] = None        # pre-smoother (3x3 block diagonal)
    Mt: Optional[sp.csr_matrix] = None       # post-smoother
    agg: Optional[np.ndarray] = None         # aggregate id per node, -1 isolated
    n_agg: int = 0
    B: Optional[np.ndarray] = None           # near-nullspace on this level
    chol: Optional[tuple] = None             # coarsest only

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def is_coarsest(self) -> bool:
        return self.chol is not None


@dataclasses.dataclass
class Hierarchy:
    levels: List[Level]
    params: AmgParams

    def sizes(self):
        return [lev.n for lev in self.levels]


# ---------------------------------------------------------------------------
# strength graph
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class StrengthGraph:
    N: int
    ptr: np.ndarray        # CSR over nodes, strong off-diagonal neighbours only
    nbr: np.ndarray
    ratio: np.ndarray      # s_IJ^2 / (s_II s_JJ) per strong link
    norm: np.ndarray       # s_IJ per strong link

    def neighbours(self, I):
        s, e = self.ptr[I], self.ptr[I + 1]
        return self.nbr[s:e], self.ratio[s:e], self.norm[s:e]


def strength_graph(A: sp.csr_matrix, b: int, eps: float) -> StrengthGraph:
    """Strong links between b x b node blocks of the scalar matrix A."""
    n = A.shape[0]
    assert n % b == 0
    N = n // b
    coo = A.tocoo()
    S2 = sp.csr_matrix((coo.data.astype(np.float64) ** 2, (coo.row // b, coo.col // b)),
                       shape=(N, N))
    S2.sum_duplicates()
    S2.sort_indices()
    s_diag = np.sqrt(S2.diagonal())
    rows = np.repeat(np.arange(N), np.diff(S2.indptr))
    cols = S2.indices
    prod = s_diag[rows] * s_diag[cols]
    strong = (rows != cols) & (S2.data >= eps * eps * prod * (1.0 - TIE_SLACK))
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(prod > 0, S2.data / prod, 0.0)
    ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows[strong], minlength=N), out=ptr[1:])
    return StrengthGraph(N, ptr, cols[strong].astype(np.int64), ratio[strong],
                         np.sqrt(S2.data[strong]))


# ---------------------------------------------------------------------------
# aggregation
# ---------------------------------------------------------------------------

def _pick_strongest(cands, ratios, agg_of):
    """Among candidate neighbours pick the strongest; ties (1e-12 relative) go
    to the lowest aggregate id."""
    rmax = max(ratios)
    best = None
    for J, r in zip(cands, ratios):
        if r >= rmax * (1.0 - TIE_SLACK):
            a = agg_of[J]
            if best is None or a < best:
                best = a
    return best


def local_qr(Ba: np.ndarray):
    """Thin QR with positive diagonal of R (unique for full column rank)."""
    Q, R = np.linalg.qr(Ba, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], R * d[:, None]


def _rank_deficient(Ba: np.ndarray) -> bool:
    if Ba.shape[0] < Ba.shape[1]:
        return True
    _, R = local_qr(Ba)
    dg = np.abs(np.diag(R))
    return not (dg.max() > 0 and dg.min() >= RANK_TOL * dg.max())


def aggregate(G: StrengthGraph, B: Optional[np.ndarray] = None, b: int = 3):
    """Greedy aggregation of the strength graph (phases 1-3 in the header).

    Returns (agg, n_agg) with agg[I] = -1 for isolated nodes.
    """
    N = G.N
    agg = [-1] * N
    ptr = G.ptr.tolist()
    nbr = G.nbr.tolist()
    ratio = G.ratio.tolist()
    isolated = [ptr[I + 1] == ptr[I] for I in range(N)]
    n_agg = 0
    # phase 1: whole strong neighbourhoods
    for I in range(N):
        if isolated[I] or agg[I] >= 0:
            continue
        nb_I = nbr[ptr[I]:ptr[I + 1]]
        if any(agg[J] >= 0 for J in nb_I):
            continue
        agg[I] = n_agg
        for J in nb_I:
            if not isolated[J]:
                agg[J] = n_agg
        n_agg += 1
    # phase 2: attach to the strongest phase-1 aggregate (snapshot)
    snap = list(agg)
    for I in range(N):
        if isolated[I] or snap[I] >= 0:
            continue
        c, r = [], []
        for k in range(ptr[I], ptr[I + 1]):
            if snap[nbr[k]] >= 0:
                c.append(nbr[k])
                r.append(ratio[k])
        if c:
            agg[I] = _pick_strongest(c, r, snap)
    agg = np.array(agg, dtype=np.int64)
    # phase 3: merge aggregates whose near-nullspace block is rank deficient
    if B is not None:
        agg, n_agg = _merge_deficient(G, agg, n_agg, B, b)
    return agg, n_agg


def _members(agg, a):
    return np.flatnonzero(agg == a)


def _local_B(B, nodes, b):
    rows = (nodes[:, None] * b + np.arange(b)[None, :]).ravel()
    return B[rows]


def _merge_deficient(G, agg, n_agg, B, b):
    alive = set(range(n_agg))
    changed = True
    while changed:
        changed = False
        for a in sorted(alive):
            if a not in alive:
                continue
            nodes = _members(agg, a)
            if not _rank_deficient(_local_B(B, nodes, b)):
                continue
            sums = {}
            for I in nodes:
                nb_I, _, nrm = G.neighbours(I)
                for J, s in zip(nb_I.tolist(), nrm.tolist()):
                    t = int(agg[J])
                    if t >= 0 and t != a:
                        sums[t] = sums.get(t, 0.0) + s
            if not sums:
                continue
            smax = max(sums.values())
            target = min(t for t, s in sums.items() if s >= smax * (1.0 - TIE_SLACK))
            agg[nodes] = target
            alive.discard(a)
            changed = True
    order = sorted(alive)
    remap = -np.ones(n_agg, dtype=np.int64)
    remap[order] = np.arange(len(order))
    out = np.where(agg >= 0, remap[np.maximum(agg, 0)], -1)
    return out, len(order)


# ---------------------------------------------------------------------------
# transfer operators
# ---------------------------------------------------------------------------

def tentative_prolongation(agg: np.ndarray, n_agg: int, B: np.ndarray, b: int):
    """P^ (n x 6 n_agg) and B_c (6 n_agg x 6) from per-aggregate thin QR."""
    N = agg.shape[0]
    n = N * b
    m = B.shape[1]
    rows_all, cols_all, vals_all = [], [], []
    Bc = np.zeros((m * n_agg, m))
    order = np.argsort(agg, kind="stable")  # node ids ascending inside each aggregate
    sorted_agg = agg[order]
    starts = np.searchsorted(sorted_agg, np.arange(n_agg))
    ends = np.searchsorted(sorted_agg, np.arange(n_agg), side="right")
    for a in range(n_agg):
        nodes = order[starts[a]:ends[a]]
        rows = (nodes[:, None] * b + np.arange(b)[None, :]).ravel()
        Q, R = local_qr(B[rows])
        rows_all.append(np.repeat(rows, m))
        cols_all.append(np.tile(np.arange(m) + m * a, rows.size))
        vals_all.append(Q.ravel())
        Bc[m * a:m * a + m] = R
    if n_agg:
        Pt = sp.csr_matrix((np.concatenate(vals_all),
                            (np.concatenate(rows_all), np.concatenate(cols_all))),
                           shape=(n, m * n_agg))
    else:
        Pt = sp.csr_matrix((n, 0))
    Pt.sort_indices()
    return Pt, Bc


def filtered_matrix(A: sp.csr_matrix, G: StrengthGraph, b: int) -> sp.csr_matrix:
    """A_F: diagonal and strong node blocks kept; weak entries lumped into the
    scalar diagonal of their row."""
    n = A.shape[0]
    N = G.N
    coo = A.tocoo()
    I = coo.row // b
    J = coo.col // b
    strong_keys = np.repeat(np.arange(N), np.diff(G.ptr)) * N + G.nbr
    strong_keys.sort()
    keys = I.astype(np.int64) * N + J
    keep = (I == J) | np.isin(keys, strong_keys, assume_unique=False)
    lump = np.bincount(coo.row[~keep], weights=coo.data[~keep], minlength=n)
    AF = sp.csr_matrix((coo.data[keep], (coo.row[keep], coo.col[keep])), shape=(n, n))
    AF = AF + sp.diags(lump)
    AF = AF.tocsr()
    AF.sort_indices()
    return AF


def smoothed_prolongation(A, G, b, Ptent, omega):
    """P = (I - omega D^{-1} A_F) P^, D the scalar diagonal of A."""
    AF = filtered_matrix(A, G, b)
    D = A.diagonal()
    if np.any(D <= 0):
        raise ValueError("matrix has a non-positive diagonal entry")
    P = Ptent - omega * (sp.diags(1.0 / D) @ (AF @ Ptent))
    P = sp.csr_matrix(P)
    P.sort_indices()
    return P


# ---------------------------------------------------------------------------
# smoothers (3x3 block diagonal)
# ---------------------------------------------------------------------------

def _diag_blocks(A: sp.csr_matrix) -> np.ndarray:
    n = A.shape[0]
    nb = n // 3
    D = np.zeros((nb, 3, 3))
    coo = A.tocoo()
    same = (coo.row // 3) == (coo.col // 3)
    np.add.at(D, (coo.row[same] // 3, coo.row[same] % 3, coo.col[same] % 3), coo.data[same])
    return D


def _block_diag_matrix(blocks: np.ndarray) -> sp.csr_matrix:
    nb = blocks.shape[0]
    M = sp.bsr_matrix((blocks, np.arange(nb), np.arange(nb + 1)), shape=(3 * nb, 3 * nb))
    return M.tocsr()


def jacobi_smoother(A: sp.csr_matrix, omega: Optional[float] = None):
    """Damped block Jacobi, M_I = omega * (A_II)^{-1} on the 3x3 diagonal blocks.

    omega None: omega = 4 / (3 lambda^) with lambda^ the power estimate of
    lambda_max(D^{-1} A) (so omega * lambda_max stays below 2 and the V-cycle
    stays positive definite)."""
    D = _diag_blocks(A)
    Dinv = np.linalg.inv(D)
    if omega is None:
        omega = 4.0 / (3.0 * power_lambda_max(A, _block_diag_matrix(Dinv)))
    M = _block_diag_matrix(omega * Dinv)
    return M, M


def spai0_smoother(A: sp.csr_matrix, omega: Optional[float] = None):
    """Damped block SPAI-0 on the 3x3 diagonal blocks.

    The undamped blocks minimise ||I - M_0 A||_F over block-diagonal M_0: row
    block I of I - M_0 A is E_I - M_I A_{I,:}, whose normal equations give
    M_I (A_{I,:} A_{I,:}^T) = A_{I,:} E_I^T = A_II^T, i.e. M_I = A_II G_I^{-1}
    with G_I = (A A^T)_II = sum_J A_IJ A_IJ^T (A symmetric).  Returns the
    pre-smoother M = omega M_0 and the post-smoother M^T, with omega as for
    block Jacobi (None: 4 / (3 lambda^), lambda^ the power estimate of
    lambda_max(M_0 A))."""
    D = _diag_blocks(A)
    G = _diag_blocks(sp.csr_matrix(A @ A.T))
    M0 = D @ np.linalg.inv(G)
    if omega is None:
        omega = 4.0 / (3.0 * power_lambda_max(A, _block_diag_matrix(M0)))
    return _block_diag_matrix(omega * M0), _block_diag_matrix(omega * np.transpose(M0, (0, 2, 1)))


def ilu0_factors(A: sp.csr_matrix):
    """Block ILU(0) of A on its own pattern of 3x3 blocks: the smoother of the
    paper's experiments (Section 3, and the NS Block rows of Tables 1-2).

    Gaussian elimination in the row-by-row (IKJ) order, in block form, that
    keeps only the blocks already present in A: for each block row i and each
    k < i in that row, L_ik = A_ik U_kk^{-1}, then A_ij -= L_ik U_kj for every
    j > k present in both row k and row i.  Returns (L, U) as CSR matrices: L
    unit block lower triangular, U block upper triangular, with (L U)_ij = A_ij
    on every block (i, j) of A's pattern (the defining property of ILU(0)).
    Plain Python loops over blocks: meant for small test matrices.
    """
    Bm = sp.bsr_matrix(A, blocksize=(3, 3))
    Bm.sort_indices()
    nb = Bm.shape[0] // 3
    ptr, idx = Bm.indptr, Bm.indices
    a = Bm.data.astype(np.float64).copy()
    where = [dict(zip(idx[ptr[i]:ptr[i + 1]].tolist(), range(ptr[i], ptr[i + 1]))) for i in range(nb)]
    diag = np.array([where[i][i] for i in range(nb)])
    for i in range(nb):
        for p in range(ptr[i], ptr[i + 1]):
            k = idx[p]
            if k >= i:
                break
            a[p] = a[p] @ np.linalg.inv(a[diag[k]])
            for q in range(diag[k] + 1, ptr[k + 1]):
                pj = where[i].get(idx[q])
                if pj is not None:
                    a[pj] -= a[p] @ a[q]
    rows = np.repeat(np.arange(nb), np.diff(ptr))
    low, up = idx < rows, idx >= rows
    def build(mask, extra_identity):
        blocks = a[mask]
        M = sp.bsr_matrix((blocks, idx[mask], np.concatenate([[0], np.cumsum(np.bincount(rows[mask], minlength=nb))])),
                          shape=A.shape)
        M = sp.csr_matrix(M)
        return M + sp.identity(A.shape[0], format="csr") if extra_identity else M
    return build(low, True), build(up, False)


def ilu0_smoother(A: sp.csr_matrix):
    """Undamped block ILU(0) relaxation, x <- x + (L U)^{-1} (f - A x), as a
    linear operator applying (L U)^{-1}.  For symmetric A the factors satisfy
    U = D L^T (D the diagonal blocks of U), so L U is symmetric and the same
    operator serves the pre- and post-sweep.

    U's diagonal blocks are full 3x3 blocks, so U is not triangular entry by
    entry; it is applied as U = D (I + D^{-1} U_s) with U_s its strictly upper
    blocks: a unit lower solve with L, the block-diagonal D^{-1}, then a unit
    upper solve with I + D^{-1} U_s (both scalar triangular)."""
    L, U = ilu0_factors(A)
    n = A.shape[0]
    D = _diag_blocks(U)
    Dinv = _block_diag_matrix(np.linalg.inv(D))
    Us = sp.csr_matrix(U - _block_diag_matrix(D))
    Ut = sp.csr_matrix(sp.identity(n, format="csr") + Dinv @ Us)

    def apply(r):
        y = spla.spsolve_triangular(L, r, lower=True, unit_diagonal=True)
        return spla.spsolve_triangular(Ut, Dinv @ y, lower=False, unit_diagonal=True)

    M = spla.LinearOperator((n, n), matvec=apply, rmatvec=apply, dtype=np.float64)
    return M, M


def greedy_block_colouring(A: sp.csr_matrix) -> np.ndarray:
    """Colour of each 3x3 block row: in increasing row order, the smallest
    colour not taken by a block neighbour already coloured.  No two coupled
    block rows share a colour."""
    Bm = sp.bsr_matrix(A, blocksize=(3, 3))
    nb = Bm.shape[0] // 3
    colour = np.full(nb, -1, dtype=np.int64)
    for i in range(nb):
        taken = {int(colour[j]) for j in Bm.indices[Bm.indptr[i]:Bm.indptr[i + 1]] if colour[j] >= 0}
        c = 0
        while c in taken:
            c += 1
        colour[i] = c
    return colour


def ilu0_multicolour_smoother(A: sp.csr_matrix):
    """Block ILU(0) in a multicolour order: block rows sorted by their greedy
    colour (stable), factored and applied in that order, then mapped back.
    Within a colour no block rows are coupled, so each triangular solve has as
    many dependent steps as there are colours."""
    colour = greedy_block_colouring(A)
    order = np.argsort(colour, kind="stable")
    perm = (3 * order[:, None] + np.arange(3)[None, :]).ravel()
    Ap = sp.csr_matrix(A[perm][:, perm])
    Ap.sort_indices()
    Mp, _ = ilu0_smoother(Ap)
    n = A.shape[0]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(n)

    def apply(r):
        return (Mp @ r[perm])[inv]

    M = spla.LinearOperator((n, n), matvec=apply, rmatvec=apply, dtype=np.float64)
    return M, M


def power_lambda_max(A: sp.csr_matrix, Dinv: sp.csr_matrix, iters: int = 30) -> float:
    """Estimate of lambda_max(M A) for a block-diagonal M (``Dinv``; D^{-1}
    for Jacobi): ``iters`` power steps from the vector x_i = (-1)^i, each
    y = M A x, lambda = ||y|| / ||x||, x = y / ||y||."""
    x = np.ones(A.shape[0])
    x[1::2] = -1.0
    lam = 0.0
    for _ in range(iters):
        y = Dinv @ (A @ x)
        ny = float(np.linalg.norm(y))
        lam = ny / float(np.linalg.norm(x))
        x = y / ny
    return lam


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------

def _constant_modes(n: int, b: int) -> np.ndarray:
    """Near-nullspace without rigid rotations: one constant vector per dof component."""
    B = np.zeros((n, b))
    for c in range(b):
        B[c::b, c] = 1.0
    return B


def build_hierarchy(A: sp.csr_matrix, coords: np.ndarray,
                    prm: Optional[AmgParams] = None) -> Hierarchy:
    prm = prm or AmgParams()
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    if prm.use_nullspace:
        B = rigid_body_modes(coords)
    else:
        B = _constant_modes(A.shape[0], 3)
    levels: List[Level] = []
    b = 3
    l = 1
    while True:
        lev = Level(A=A, b=b, eps=prm.eps_strong * prm.eps_decay ** (l - 1), B=B)
        levels.append(lev)
        if A.shape[0] <= prm.coarse_enough or l >= prm.max_levels:
            break
        G = strength_graph(A, b, lev.eps)
        agg, n_agg = aggregate(G, B, b)
        m = B.shape[1]
        if n_agg == 0 or m * n_agg > 0.9 * A.shape[0]:
            break
        Ptent, Bc = tentative_prolongation(agg, n_agg, B, b)
        P = smoothed_prolongation(A, G, b, Ptent, prm.omega_p)
        R = sp.csr_matrix(P.T)
        R.sort_indices()
        Ac = sp.csr_matrix(R @ A @ P)
        Ac.sort_indices()
        lev.P, lev.R, lev.Ptent, lev.agg, lev.n_agg = P, R, Ptent, agg, n_agg
        below = prm.smoother_levels is not None and l > prm.smoother_levels
        if prm.smoother == "jacobi" or (below and prm.smoother.startswith("ilu0")):
            lev.M, lev.Mt = jacobi_smoother(A, prm.omega_j)
        elif prm.smoother == "spai0":
            lev.M, lev.Mt = spai0_smoother(A, prm.omega_j)
        elif prm.smoother == "ilu0":
            lev.M, lev.Mt = ilu0_smoother(A)
        elif prm.smoother == "ilu0_mc":
            lev.M, lev.Mt = ilu0_multicolour_smoother(A)
        else:
            raise ValueError(prm.smoother)
        A, B, b = Ac, Bc, m
        l += 1
    last = levels[-1]
    last.chol = sla.cho_factor(last.A.toarray(), lower=True)
    return Hierarchy(levels, prm)


def smoother_spectral_radius(lev: Level, iters: int = 30) -> float:
    """Estimate of lambda_max(M A) by power iteration from the all-ones vector."""
    x = np.ones(lev.n)
    lam = 0.0
    for _ in range(iters):
        y = lev.M @ (lev.A @ x)
        lam = float(np.linalg.norm(y) / np.linalg.norm(x))
        x = y / np.linalg.norm(y)
    return lam
