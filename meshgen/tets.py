"""Linear (P1) tetrahedral elasticity on a Kuhn-split structured grid.

The paper's two measured matrices (a connecting rod and a solid hook, Section
4) come from unstructured P1 tetrahedral meshes that are not available.  These
stand-ins give the same element type, block structure and size class: a unit
cube of (nn-1)^3 grid cells, each split into six tetrahedra along its main
diagonal (Kuhn split: one tetrahedron per ordering of the three axes, walking
from corner (0,0,0) to corner (1,1,1)), isotropic material with E = 1, clamped
at x = 0, body force (0, 0, -1).

With that split every edge joins two grid nodes whose offsets are all >= 0 or
all <= 0, so an interior node couples to 15 nodes (itself, 7 offsets in
{0,1}^3 and their negatives).  Node numbering, unknown ordering, clamping and
the block CSR output follow the hexahedral generator.
"""
from __future__ import annotations

import itertools

import numpy as np

from .elasticity import Problem, _node_ijk


def p1_element_stiffness(X: np.ndarray, nu: float, E: float = 1.0) -> np.ndarray:
    """12x12 stiffness of a linear tetrahedron with vertices X[4, 3].

    With g_a the (constant) gradient of vertex a's barycentric coordinate and
    V the volume, block (a, b) is V (lam g_a g_b^T + mu g_b g_a^T + mu (g_a.g_b) I):
    row (a, i) tests with N_a e_i, column (b, j) is the trial field N_b e_j.
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    J = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)  # columns: edge vectors
    V = abs(np.linalg.det(J)) / 6.0
    Jinv = np.linalg.inv(J)
    g = np.zeros((4, 3))
    g[1:] = Jinv          # grad of xi_k = row k of J^{-1}
    g[0] = -Jinv.sum(axis=0)
    K = np.zeros((12, 12))
    for a in range(4):
        for b in range(4):
            K[3 * a:3 * a + 3, 3 * b:3 * b + 3] = V * (lam * np.outer(g[a], g[b]) + mu * np.outer(g[b], g[a])
                                                     + mu * (g[a] @ g[b]) * np.eye(3))
    return K


def kuhn_tets():
    """The six tetrahedra of a unit cell as lists of corner offsets (di, dj, dk)."""
    tets = []
    for perm in itertools.permutations(range(3)):
        v = [0, 0, 0]
        verts = [tuple(v)]
        for ax in perm:
            v[ax] += 1
            verts.append(tuple(v))
        tets.append(verts)
    return tets


def assemble_tets(nn: int, nu: float = 0.3, clamp_x0: bool = True):
    """Assemble the block stiffness of the Kuhn-split unit cube with nn^3 nodes.

    Returns ``(row_ptr, col, val, coords, fixed, tet_nodes, tet_volume)``.
    """
    n = nn - 1
    h = 1.0 / n
    nb = nn ** 3
    i, j, k = _node_ijk(n, n, n)
    fixed = (i == 0) if clamp_x0 else np.zeros(nb, dtype=bool)
    px, py = nn, nn * nn

    # 15-point block pattern; offsets in (dk, dj, di) order keep columns sorted
    offsets = [(di, dj, dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)
               if min(di, dj, dk) >= 0 or max(di, dj, dk) <= 0]
    slot = {o: s for s, o in enumerate(offsets)}
    centre = slot[(0, 0, 0)]
    node = np.arange(nb, dtype=np.int64)
    valid = np.zeros((nb, len(offsets)), dtype=bool)
    colmat = np.zeros((nb, len(offsets)), dtype=np.int64)
    for s, (di, dj, dk) in enumerate(offsets):
        ok = ((i + di >= 0) & (i + di <= n) & (j + dj >= 0) & (j + dj <= n)
              & (k + dk >= 0) & (k + dk <= n))
        J = node + di + px * dj + py * dk
        if s != centre:
            Jc = np.where(ok, J, 0)
            ok = ok & ~fixed & ~fixed[Jc]
        valid[:, s] = ok
        colmat[:, s] = J
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    pos = row_ptr[:-1, None] + np.cumsum(valid, axis=1) - valid
    col = np.empty(int(row_ptr[-1]), dtype=np.int64)
    col[pos[valid]] = colmat[valid]
    val = np.zeros((col.shape[0], 3, 3), dtype=np.float64)

    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = (ci.transpose(2, 1, 0).ravel() + px * cj.transpose(2, 1, 0).ravel()
            + py * ck.transpose(2, 1, 0).ravel()).astype(np.int64)
    tet_nodes = []
    vol = h ** 3 / 6.0
    for verts in kuhn_tets():
        Ke = p1_element_stiffness(h * np.asarray(verts, dtype=np.float64), nu)
        gl = [base + v[0] + px * v[1] + py * v[2] for v in verts]
        tet_nodes.append(np.stack(gl, axis=1))
        for a in range(4):
            I = gl[a]
            for b in range(4):
                off = tuple(int(x) for x in np.subtract(verts[b], verts[a]))
                s = slot[off]
                ok = valid[I, s]
                # one cell per (I, slot) for a fixed tetrahedron type and local pair
                val[pos[I[ok], s]] += Ke[3 * a:3 * a + 3, 3 * b:3 * b + 3][None, :, :]
    val[pos[fixed, centre]] = np.eye(3)
    coords = np.stack([i * h, j * h, k * h], axis=1).astype(np.float64)
    return (row_ptr.astype(np.int32), col.astype(np.int32), val, coords, fixed,
            np.concatenate(tet_nodes, axis=0), vol)


def tet_cube(nn: int, nu: float = 0.3, name: str | None = None) -> Problem:
    """Kuhn-split P1 unit cube with nn^3 nodes, clamped at x = 0, body force (0,0,-1)."""
    row_ptr, col, val, coords, fixed, tets, vol = assemble_tets(nn, nu)
    nb = coords.shape[0]
    w = np.bincount(tets.ravel(), minlength=nb) * (vol / 4.0)  # int N_a dV
    b = np.zeros((nb, 3))
    b[:, 2] = -w
    b[fixed] = 0.0
    n = nn - 1
    return Problem(name or f"tets{nn}", row_ptr, col, val, coords, b.ravel(), (n, n, n),
                   (1.0 / n,) * 3, nu, fixed)


def rod_standin() -> Problem:
    """Size stand-in for the paper's connecting rod: 30^3 nodes, 81,000 unknowns."""
    return tet_cube(30, name="tets30_rod_standin")


def hook_standin() -> Problem:
    """Size stand-in for the paper's solid hook: 27^3 nodes, 59,049 unknowns."""
    return tet_cube(27, name="tets27_hook_standin")
