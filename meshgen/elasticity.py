"""Q1 hexahedral linear-elasticity assembly straight into 3x3 node blocks.

The paper's model problems are 3D elasticity systems whose matrices have
natural 3x3 blocks, one per pair of mesh nodes (Section 2, discussion of
Fig. 1).  The paper's own matrices (a connecting rod and a solid hook,
Section 4) are not available, so the workloads here are synthetic structured
boxes of trilinear hexahedra with the same block structure:

* nodes are numbered ``id = i + (nx+1)*(j + (ny+1)*k)`` (x fastest), elements
  the same way over ``nx*ny*nz``;
* isotropic material, ``lambda = E nu / ((1+nu)(1-2nu))``,
  ``mu = E / (2(1+nu))``, integrated with 2x2x2 Gauss-Legendre points;
* unknowns are node-major (u_x, u_y, u_z of node 0, then node 1, ...);
* a clamped node keeps only an identity diagonal block: its block row and block
  column are removed from the pattern and its right-hand side entry is zero.

The block matrix is returned as int32 ``row_ptr[nb+1]``, int32 ``col[nnzb]``
(sorted within each row, diagonal always present) and float64
``val[nnzb, 3, 3]`` (row-major blocks).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Problem:
    """One elasticity system in 3x3-block CSR form plus its node coordinates."""

    name: str
    row_ptr: np.ndarray  # int32 [nb+1]
    col: np.ndarray      # int32 [nnzb]
    val: np.ndarray      # float64 [nnzb, 3, 3]
    coords: np.ndarray   # float64 [nb, 3]
    b: np.ndarray        # float64 [3*nb] or [3*nb, k]
    dims: tuple          # (nx, ny, nz) elements
    spacing: tuple       # (hx, hy, hz)
    nu: float
    fixed: np.ndarray    # bool [nb], clamped nodes

    @property
    def nb(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def n(self) -> int:
        return 3 * self.nb

    @property
    def nnzb(self) -> int:
        return int(self.col.shape[0])

    def csr(self) -> sp.csr_matrix:
        return bsr_to_csr(self.row_ptr, self.col, self.val)


# ---------------------------------------------------------------------------
# element stiffness
# ---------------------------------------------------------------------------

def _local_signs():
    # local node a = ia + 2*ja + 4*ka, reference coordinate sign 2*i-1
    s = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                  for a in range(8)], dtype=np.float64)
    return s


def q1_element_stiffness(hx: float, hy: float, hz: float, nu: float,
                         E: float = 1.0) -> np.ndarray:
    """24x24 stiffness of an axis-aligned hx*hy*hz trilinear brick.

    Dof order is node-major over the 8 local nodes (local node
    ``ia + 2 ja + 4 ka``), components x, y, z.  Voigt strain order is
    (xx, yy, zz, yz, xz, xy) with engineering shears.
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    s = _local_signs()
    g = 1.0 / np.sqrt(3.0)
    detJ = hx * hy * hz / 8.0
    K = np.zeros((24, 24))
    for gx in (-g, g):
        for gy in (-g, g):
            for gz in (-g, g):
                # derivatives of N_a = (1+sx xi)(1+sy eta)(1+sz zeta)/8
                dxi = s[:, 0] * (1 + s[:, 1] * gy) * (1 + s[:, 2] * gz) / 8.0
                deta = s[:, 1] * (1 + s[:, 0] * gx) * (1 + s[:, 2] * gz) / 8.0
                dzeta = s[:, 2] * (1 + s[:, 0] * gx) * (1 + s[:, 1] * gy) / 8.0
                dx = dxi * 2.0 / hx
                dy = deta * 2.0 / hy
                dz = dzeta * 2.0 / hz
                B = np.zeros((6, 24))
                B[0, 0::3] = dx
                B[1, 1::3] = dy
                B[2, 2::3] = dz
                B[3, 1::3] = dz
                B[3, 2::3] = dy
                B[4, 0::3] = dz
                B[4, 2::3] = dx
                B[5, 0::3] = dy
                B[5, 1::3] = dx
                K += B.T @ D @ B * detJ
    return 0.5 * (K + K.T)


# ---------------------------------------------------------------------------
# global assembly
# ---------------------------------------------------------------------------

def _node_ijk(nx, ny, nz):
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                          indexing="ij")
    # node id order: x fastest
    i = i.transpose(2, 1, 0).ravel()
    j = j.transpose(2, 1, 0).ravel()
    k = k.transpose(2, 1, 0).ravel()
    return i.astype(np.int64), j.astype(np.int64), k.astype(np.int64)


def _connectivity(nx, ny, nz):
    ei, ej, ek = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ei = ei.transpose(2, 1, 0).ravel().astype(np.int64)
    ej = ej.transpose(2, 1, 0).ravel().astype(np.int64)
    ek = ek.transpose(2, 1, 0).ravel().astype(np.int64)
    px, py = nx + 1, (nx + 1) * (ny + 1)
    conn = np.empty((ei.size, 8), dtype=np.int64)
    for a in range(8):
        ia, ja, ka = a & 1, (a >> 1) & 1, (a >> 2) & 1
        conn[:, a] = (ei + ia) + px * (ej + ja) + py * (ek + ka)
    return conn, (ei, ej, ek)


def assemble_box(nx: int, ny: int, nz: int, hx: float, hy: float, hz: float,
                 nu: float, E_elem: Optional[np.ndarray] = None,
                 clamp_x0: bool = True):
    """Assemble the block stiffness matrix of an nx*ny*nz brick mesh.

    Returns ``(row_ptr, col, val, coords, fixed)``.  ``E_elem`` gives the Young
    modulus per element (element order, x fastest); default 1.
    """
    nb = (nx + 1) * (ny + 1) * (nz + 1)
    ne = nx * ny * nz
    if E_elem is None:
        E_elem = np.ones(ne)
    E_elem = np.asarray(E_elem, dtype=np.float64)
    assert E_elem.shape == (ne,)
    Ke = q1_element_stiffness(hx, hy, hz, nu)
    i, j, k = _node_ijk(nx, ny, nz)
    fixed = (i == 0) if clamp_x0 else np.zeros(nb, dtype=bool)
    px, py = nx + 1, (nx + 1) * (ny + 1)

    # 27-point block pattern, offsets ordered (dk, dj, di) so columns increase
    valid = np.zeros((nb, 27), dtype=bool)
    colmat = np.zeros((nb, 27), dtype=np.int64)
    node = np.arange(nb, dtype=np.int64)
    for s in range(27):
        dk, dj, di = s // 9 - 1, (s // 3) % 3 - 1, s % 3 - 1
        ok = ((i + di >= 0) & (i + di <= nx) & (j + dj >= 0) & (j + dj <= ny)
              & (k + dk >= 0) & (k + dk <= nz))
        J = node + di + px * dj + py * dk
        if s != 13:
            Jc = np.where(ok, J, 0)
            ok = ok & ~fixed & ~fixed[Jc]
        valid[:, s] = ok
        colmat[:, s] = J
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnzb = int(row_ptr[-1])
    pos = row_ptr[:-1, None] + np.cumsum(valid, axis=1) - valid  # slot position
    col = np.empty(nnzb, dtype=np.int64)
    col[pos[valid]] = colmat[valid]
    val = np.zeros((nnzb, 3, 3), dtype=np.float64)

    conn, _ = _connectivity(nx, ny, nz)
    for a in range(8):
        ia, ja, ka = a & 1, (a >> 1) & 1, (a >> 2) & 1
        I = conn[:, a]
        for b in range(8):
            ib, jb, kb = b & 1, (b >> 1) & 1, (b >> 2) & 1
            s = (kb - ka + 1) * 9 + (jb - ja + 1) * 3 + (ib - ia + 1)
            ok = valid[I, s]
            blk = Ke[3 * a:3 * a + 3, 3 * b:3 * b + 3]
            idx = pos[I[ok], s]
            # each element owns a distinct (I, J) for a fixed local pair (a, b)
            val[idx] += E_elem[ok, None, None] * blk[None, :, :]
    dpos = pos[fixed, 13]
    val[dpos] = np.eye(3)
    coords = np.stack([i * hx, j * hy, k * hz], axis=1).astype(np.float64)
    return (row_ptr.astype(np.int32), col.astype(np.int32), val, coords, fixed)


def _body_force(nx, ny, nz, hx, hy, hz, fixed, force=(0.0, 0.0, -1.0)):
    nb = fixed.shape[0]
    conn, _ = _connectivity(nx, ny, nz)
    w = np.bincount(conn.ravel(), minlength=nb) * (hx * hy * hz / 8.0)
    b = np.zeros((nb, 3))
    for c in range(3):
        b[:, c] = force[c] * w
    b[fixed] = 0.0
    return b.ravel()


def _tip_load(nx, ny, nz, hx, hy, hz, fixed, total=(0.0, 0.0, -1.0)):
    """Total force ``total`` spread over the face x = nx*hx with weights int N_a dA."""
    nb = fixed.shape[0]
    px, py = nx + 1, (nx + 1) * (ny + 1)
    area = (ny * hy) * (nz * hz)
    w = np.zeros(nb)
    for fj in range(ny):
        for fk in range(nz):
            for dj in (0, 1):
                for dk in (0, 1):
                    w[nx + px * (fj + dj) + py * (fk + dk)] += hy * hz / 4.0
    b = np.zeros((nb, 3))
    for c in range(3):
        b[:, c] = total[c] * w / area
    b[fixed] = 0.0
    return b.ravel()


def bsr_to_csr(row_ptr, col, val) -> sp.csr_matrix:
    """Unblock a 3x3 block CSR matrix into scalar CSR, dropping exact zeros."""
    nb = len(row_ptr) - 1
    A = sp.bsr_matrix((np.asarray(val), np.asarray(col), np.asarray(row_ptr)),
                      shape=(3 * nb, 3 * nb)).tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    return A


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def _box_problem(name, nx, ny, nz, hx, hy, hz, nu, E_elem, load):
    rp, col, val, coords, fixed = assemble_box(nx, ny, nz, hx, hy, hz, nu, E_elem)
    if load == "body":
        b = _body_force(nx, ny, nz, hx, hy, hz, fixed)
    elif load == "tip":
        b = _tip_load(nx, ny, nz, hx, hy, hz, fixed)
    else:
        b = load
    return Problem(name, rp, col, val, coords, b, (nx, ny, nz), (hx, hy, hz), nu, fixed)


def cube_c1(n: int = 10, nu: float = 0.3) -> Problem:
    """Unit cube of n^3 bricks, E = 1, clamped at x = 0, body force (0,0,-1)."""
    h = 1.0 / n
    return _box_problem(f"cube{n}", n, n, n, h, h, h, nu, None, "body")


def cube_lognormal(n: int = 64, seed: int = 0, nu: float = 0.3) -> Problem:
    """Unit cube, E_e = exp(Z_e), Z ~ N(0,1) i.i.d. in element order."""
    h = 1.0 / n
    Z = np.random.default_rng(seed).standard_normal(n ** 3)
    return _box_problem(f"cube{n}_lognormal", n, n, n, h, h, h, nu, np.exp(Z), "body")


def cube_inclusions(n: int = 96, n_incl: int = 100, radius_elems: float = 6.0,
                    E_incl: float = 1000.0, seed: int = 1, nu: float = 0.3) -> Problem:
    """Unit cube with stiff spherical inclusions (by element centroid)."""
    h = 1.0 / n
    centres = np.random.default_rng(seed).uniform(0.0, 1.0, size=(n_incl, 3))
    _, (ei, ej, ek) = _connectivity(n, n, n)
    cx, cy, cz = (ei + 0.5) * h, (ej + 0.5) * h, (ek + 0.5) * h
    inside = np.zeros(n ** 3, dtype=bool)
    r2 = (radius_elems * h) ** 2
    for c in centres:
        inside |= (cx - c[0]) ** 2 + (cy - c[1]) ** 2 + (cz - c[2]) ** 2 <= r2
    E = np.where(inside, E_incl, 1.0)
    return _box_problem(f"cube{n}_inclusions", n, n, n, h, h, h, nu, E, "body")


def cube_multi_rhs(n: int = 48, k: int = 32, seed: int = 2, nu: float = 0.3) -> Problem:
    """Unit cube, E = 1, k load cases with N(0,1) entries per dof (clamped dofs 0)."""
    h = 1.0 / n
    rp, col, val, coords, fixed = assemble_box(n, n, n, h, h, h, nu)
    B = np.random.default_rng(seed).standard_normal((3 * len(coords), k))
    B[np.repeat(fixed, 3)] = 0.0
    return Problem(f"cube{n}_rhs{k}", rp, col, val, coords, B, (n, n, n), (h, h, h), nu, fixed)


def batch_cubes(count: int = 64, lo: int = 8, hi: int = 32, seed: int = 3) -> List[Problem]:
    """``count`` unit cubes with edge sizes drawn uniformly from {lo..hi} elements."""
    edges = np.random.default_rng(seed).integers(lo, hi + 1, size=count)
    return [cube_c1(int(e)) for e in edges]


def beam(nx: int = 256, ny: int = 32, nz: int = 32, nu: float = 0.45) -> Problem:
    """Beam of length nx/ny (aspect 4:1:1 bricks), clamped at x = 0, tip load."""
    hy = hz = 1.0 / ny
    hx = 4.0 * hy
    return _box_problem(f"beam{nx}x{ny}x{nz}", nx, ny, nz, hx, hy, hz, nu, None, "tip")


def training_beams() -> List[Problem]:
    """The three small beams the learned smoother is trained on."""
    return [beam(32, 4, 4), beam(64, 8, 8), beam(128, 16, 16)]


def named_problem(name: str) -> Problem:
    """Workloads by name: the five configurations and small variants."""
    table = {
        "cube10": lambda: cube_c1(10),
        "cube64_lognormal": lambda: cube_lognormal(64, 0),
        "cube96_inclusions": lambda: cube_inclusions(96),
        "cube48_rhs32": lambda: cube_multi_rhs(48, 32),
        "beam256x32x32": lambda: beam(256, 32, 32),
    }
    if name in table:
        return table[name]()
    raise KeyError(name)
