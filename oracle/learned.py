"""Learned per-node smoother blocks (oracle; test infrastructure only).

The paper's method relaxes with damped block Jacobi on the 3x3 diagonal
blocks (Section 3: block-valued smoothers; Algorithm 2 smooths before and
after the coarse correction).  The paper has no learned part; this module is
the plain FP64 definition of the learned variant that replaces the level-1
block-Jacobi blocks M_i = omega_J A_ii^{-1}, written from these choices:

Slots.  For node i and a node j whose block A_ij is stored, the slot of j is
    k(i, j) = 9 (sx + 1) + 3 (sy + 1) + (sz + 1),
with s the sign (-1, 0, 1) of each coordinate difference x_j - x_i; a
difference of at most 1e-8 times the largest bounding-box extent counts as 0.
Slot 13 is the node itself.  Two neighbours of one node in one slot are
rejected (a node of a hexahedral grid has at most one neighbour per slot).

Features of node i (90 values, scale free):
    phi_i = [ D_i / d_i (row-major, 9) ,  diag(A_ij) / d_i at slot k(i, j) (27 x 3) ],
with D_i = A_ii and d_i = ||D_i||_F; unoccupied slots are 0.

Network (10,374 parameters, flat vector in this order):
    W1 [90][64], b1 [64], W2 [64][64], b2 [64], W3 [64][6], b3 [6]
    h1 = relu(W1^T phi + b1),  h2 = relu(W2^T h1 + b2),  g = W3^T h2 + b3.

Smoother block (M_i = L_i L_i^T its Cholesky factorisation):
    S_i = L_i (I + X_i) L_i^T,   X_i = sym(c * tanh(g_i)),
    sym(u) = [[u0, u3, u4], [u3, u1, u5], [u4, u5, u2]],  c = (.25, .25, .25, .05, .05, .05),
used in place of M_i for every level-1 relaxation x += S (f - A x).  S is
symmetric block diagonal, so the V-cycle stays symmetric and plain CG applies.
With W3 = 0 and b3 = 0, X = 0 and S = M: the block-Jacobi method.

Safe band.  With Lam = 4 / (3 omega_J) (the damping's estimate of
lambda_max(D^{-1} A), so A <= Lam D), a symmetric block-diagonal S with
    0 < S_i < (2 KAPPA / Lam) D_i^{-1} = 1.5 KAPPA M_i      (Loewner order)
gives 2 S^{-1} - A >= Lam (1/KAPPA - 1) D > 0: the relaxation contracts the
error in the energy norm (KAPPA = 0.9 leaves room for Lam being a slight
underestimate).  By Gershgorin every eigenvalue of X_i lies in
(-0.35, 0.35), so I + X_i lies in (0.65, 1.35) and S_i inside the band for
any network output: the learned smoother can never diverge.

Training loss (two-grid energy).  For an error e, r = A e, smoothed error
w = e - S r, then the coarse-grid correction y = (I - Pi) w with
Pi = P V_2(R A .) (V_2 the coarse V-cycle from level 2):
    l(e) = y^T A y / (e^T A e);   a batch averages l over its errors.
Because V_2 is symmetric, (I - Pi)^T A = A (I - Pi), hence
    dl/dw = 2 A (I - Pi) y / (e^T A e),   dl/dS_i = -(dl/dw)_i r_i^T,
dl/dX_i = L_i^T (dl/dS_i) L_i, dl/dg_i = c (1 - tanh^2 g_i) sym^T(dl/dX_i),
and back-propagation through the two ReLU layers gives the parameter gradient.  Adam (Kingma and Ba, 2015) with
bias correction updates the parameters.

Training errors come from the method itself: random errors after c stationary
V-cycle steps e <- e - V(A e) of the block-Jacobi method.

Pinned by: central finite differences of the loss against the gradient;
zero last layer = block Jacobi; a hand-built network whose output is a known
constant (closed form S_i = L_i (I + X) L_i^T); the band against eigenvalues
of the generalised problem S v = mu M v; Adam's first step in closed form;
slot geometry on a brick grid.  The benefit of the trained network is empirical
(parity unpinned): it is measured, not derived.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

from .setup import Hierarchy, _diag_blocks

N_FEAT = 90
N_HID = 64
N_OUT = 6
SHAPES = [("W1", (N_FEAT, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 10,374
KAPPA = 0.9
SYM_INDEX = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
SPREAD = np.array([0.25, 0.25, 0.25, 0.05, 0.05, 0.05])


def unpack(theta: np.ndarray) -> dict:
    """Views of the flat parameter vector by name."""
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters, got {theta.shape}")
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def sym(g: np.ndarray) -> np.ndarray:
    """(n, 6) -> (n, 3, 3) symmetric blocks."""
    G = np.zeros((g.shape[0], 3, 3))
    for k, (a, b) in enumerate(SYM_INDEX):
        G[:, a, b] = g[:, k]
        G[:, b, a] = g[:, k]
    return G


def sym_adjoint(U: np.ndarray) -> np.ndarray:
    """Adjoint of ``sym``: (n, 3, 3) -> (n, 6)."""
    out = np.zeros((U.shape[0], 6))
    for k, (a, b) in enumerate(SYM_INDEX):
        out[:, k] = U[:, a, b] if a == b else U[:, a, b] + U[:, b, a]
    return out


# ---------------------------------------------------------------------------
# neighbourhood and features
# ---------------------------------------------------------------------------

def neighbour_slots(row_ptr, col, coords) -> np.ndarray:
    """Slot k(i, j) of every stored block (in storage order)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    coords = np.asarray(coords, dtype=np.float64)
    nb = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(nb), np.diff(row_ptr))
    extent = float((coords.max(axis=0) - coords.min(axis=0)).max()) if nb else 0.0
    tau = 1e-8 * extent
    d = coords[col] - coords[rows]
    s = np.where(d > tau, 1, np.where(d < -tau, -1, 0))
    slots = 9 * (s[:, 0] + 1) + 3 * (s[:, 1] + 1) + (s[:, 2] + 1)
    key = rows * 27 + slots
    if np.unique(key).shape[0] != key.shape[0]:
        raise ValueError("two neighbours of one node fall into the same slot")
    return slots.astype(np.int64)


@dataclasses.dataclass
class LearnedLevel:
    """What the learned smoother needs of the finest level."""
    phi: np.ndarray         # (nb, 90) features
    D: np.ndarray           # (nb, 3, 3) diagonal blocks
    Dnorm: np.ndarray       # (nb,) Frobenius norms
    Mblk: np.ndarray        # (nb, 3, 3) block-Jacobi blocks omega_J D^-1
    Lchol: np.ndarray       # (nb, 3, 3) lower Cholesky factors of Mblk
    omega: float
    A: sp.csr_matrix        # scalar A_1

    @property
    def nb(self) -> int:
        return self.D.shape[0]


def features(row_ptr, col, val, coords) -> np.ndarray:
    """phi (nb, 90) from the stored blocks of A_1 (val: (nnzb, 3, 3))."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    nb = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(nb), np.diff(row_ptr))
    slots = neighbour_slots(row_ptr, col, coords)
    on_diag = rows == col
    D = np.zeros((nb, 3, 3))
    D[rows[on_diag]] = val[on_diag]
    dn = np.sqrt((D * D).sum(axis=(1, 2)))
    phi = np.zeros((nb, N_FEAT))
    phi[:, :9] = (D / dn[:, None, None]).reshape(nb, 9)
    for c in range(3):
        phi[rows, 9 + 3 * slots + c] = val[:, c, c] / dn[rows]
    return phi


def learned_level(h: Hierarchy, row_ptr, col, val, coords) -> LearnedLevel:
    lev = h.levels[0]
    D = _diag_blocks(lev.A)
    Mblk = _diag_blocks(lev.M)
    omega = float(np.einsum("iab,iba->", Mblk, D)) / (3 * D.shape[0])   # M_i D_i = omega I
    return LearnedLevel(features(row_ptr, col, val, coords), D, np.sqrt((D * D).sum(axis=(1, 2))),
                        Mblk, np.linalg.cholesky(Mblk), omega, lev.A)


# ---------------------------------------------------------------------------
# network and smoother blocks
# ---------------------------------------------------------------------------

def mlp_forward(theta: np.ndarray, phi: np.ndarray):
    p = unpack(theta)
    z1 = phi @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    g = h2 @ p["W3"] + p["b3"]
    return g, (phi, z1, h1, z2, h2)


def mlp_backward(theta: np.ndarray, cache, dg: np.ndarray) -> np.ndarray:
    """Gradient of sum_i dg_i . g_i with respect to theta."""
    p = unpack(theta)
    phi, z1, h1, z2, h2 = cache
    dW3 = h2.T @ dg
    db3 = dg.sum(axis=0)
    dz2 = (dg @ p["W3"].T) * (z2 > 0.0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * (z1 > 0.0)
    dW1 = phi.T @ dz1
    db1 = dz1.sum(axis=0)
    return pack({"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": db3})


def _pos_def3(S: np.ndarray) -> np.ndarray:
    """Leading principal minors of each 3x3 symmetric block all positive."""
    m1 = S[:, 0, 0]
    m2 = S[:, 0, 0] * S[:, 1, 1] - S[:, 0, 1] * S[:, 1, 0]
    m3 = np.linalg.det(S)
    return (m1 > 0.0) & (m2 > 0.0) & (m3 > 0.0)


def in_band(L: LearnedLevel, S: np.ndarray) -> np.ndarray:
    """0 < S_i < 1.5 KAPPA M_i for each node."""
    return _pos_def3(S) & _pos_def3(1.5 * KAPPA * L.Mblk - S)


def smoother_blocks(L: LearnedLevel, theta: np.ndarray, return_parts: bool = False):
    """S (nb, 3, 3) = L_i (I + X_i) L_i^T."""
    g, cache = mlp_forward(theta, L.phi)
    t = np.tanh(g)
    T = np.eye(3)[None] + sym(SPREAD * t)
    S = np.einsum("iab,ibc,idc->iad", L.Lchol, T, L.Lchol)
    if return_parts:
        return S, (cache, t)
    return S


def block_apply(S: np.ndarray, r: np.ndarray) -> np.ndarray:
    return np.einsum("iab,ib->ia", S, np.asarray(r).reshape(-1, 3)).reshape(-1)


# ---------------------------------------------------------------------------
# the method with learned blocks, training loss and optimizer
# ---------------------------------------------------------------------------

def vcycle_blocks(h: Hierarchy, S: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Algorithm 2 with the level-1 relaxations using the blocks S (coarser
    levels keep block Jacobi)."""
    from .solve import vcycle
    lev = h.levels[0]
    if lev.is_coarsest:
        return vcycle(h, f)
    x = block_apply(S, f)
    for _ in range(h.params.npre - 1):
        x = x + block_apply(S, f - lev.A @ x)
    r = f - lev.A @ x
    x = x + lev.P @ vcycle(h, lev.R @ r, 1)
    for _ in range(h.params.npost):
        x = x + block_apply(S, f - lev.A @ x)
    return x


def coarse_correction(h: Hierarchy, e: np.ndarray) -> np.ndarray:
    """(I - Pi) e = e - P V_2(R A e)."""
    from .solve import vcycle
    lev = h.levels[0]
    return e - lev.P @ vcycle(h, lev.R @ (lev.A @ e), 1)


def loss_and_grad(h: Hierarchy, L: LearnedLevel, theta: np.ndarray, E: np.ndarray):
    """Mean two-grid energy ratio over the columns of E (n x k) and its gradient."""
    E = np.asarray(E, dtype=np.float64)
    if E.ndim == 1:
        E = E[:, None]
    S, (cache, t) = smoother_blocks(L, theta, return_parts=True)
    A = L.A
    k = E.shape[1]
    total = 0.0
    U = np.zeros((L.nb, 3, 3))
    for j in range(k):
        e = E[:, j]
        r = A @ e
        den = float(e @ r)
        w = e - block_apply(S, r)
        y = coarse_correction(h, w)
        total += float(y @ (A @ y)) / den
        dl_dw = (2.0 / den) * (A @ coarse_correction(h, y))
        # w = e - S r:  dl/dS_i = -(dl/dw)_i r_i^T
        U -= np.einsum("ia,ib->iab", dl_dw.reshape(-1, 3), r.reshape(-1, 3))
    U /= k
    dX = np.einsum("iba,ibc,icd->iad", L.Lchol, U, L.Lchol)      # L^T U L
    dg = SPREAD * (1.0 - t * t) * sym_adjoint(dX)
    return total / k, mlp_backward(theta, cache, dg)


def loss_only(h: Hierarchy, L: LearnedLevel, theta: np.ndarray, E: np.ndarray) -> float:
    E = np.asarray(E, dtype=np.float64)
    if E.ndim == 1:
        E = E[:, None]
    S = smoother_blocks(L, theta)
    total = 0.0
    for j in range(E.shape[1]):
        e = E[:, j]
        r = L.A @ e
        y = coarse_correction(h, e - block_apply(S, r))
        total += float(y @ (L.A @ y)) / float(e @ r)
    return total / E.shape[1]


def adam_step(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def training_errors(h: Hierarchy, E0: np.ndarray, cycles: int,
                    precond: Optional[Callable[[np.ndarray], np.ndarray]] = None) -> np.ndarray:
    """Columns of E0 after ``cycles`` stationary steps e <- e - V(A e)."""
    from .solve import vcycle
    A = h.levels[0].A
    if precond is None:
        precond = lambda v: vcycle(h, v)  # noqa: E731
    E = np.array(E0, dtype=np.float64, copy=True)
    if E.ndim == 1:
        E = E[:, None]
    for j in range(E.shape[1]):
        e = E[:, j]
        for _ in range(cycles):
            e = e - precond(A @ e)
        E[:, j] = e
    return E
