"""V-cycle and (flexible) preconditioned CG in scalar CSR (oracle; test
infrastructure only).

V-cycle (Algorithm 2 of the paper, one cycle per preconditioner application as
Section 2 describes, zero initial guess on every level):

    V_l(f):  x = M_l f                          (pre-smoothing from x = 0)
             repeat npre-1 times: x += M_l (f - A_l x)
             r = f - A_l x;  f_c = R_l r        (residual, restriction)
             x_c = V_{l+1}(f_c)  (A_L^{-1} f_c at the coarsest level)
             x = x + P_l x_c                    (undamped correction)
             repeat npost times: x += M_l^T (f - A_l x)
             return x

Conjugate gradients with this preconditioner (Section 4: CG, relative residual
1e-8): x_0 given or 0, r = b - A x_0, z = V(r), p = z; each iteration
q = A p, alpha = r.z / p.q, x += alpha p, r -= alpha q; when ||r|| <= tol ||b||
the true residual b - A x is recomputed and accepted if it also meets the
target, otherwise CG restarts from it (at most ``max_restarts`` times);
z = V(r), beta = r_new.z_new / r_old.z_old (flexible variant:
beta = r_new.(z_new - z_old) / r_old.z_old), p = z + beta p.  The iteration
count is the number of products A p.

Pinned by: the V-cycle's dense operator against the recursive closed form
B_l = (I - E_l) A_l^{-1}, E_l = (I - M_l^T A_l)(I - P_l B_{l+1} R_l A_l)(I - M_l A_l),
its symmetry and positivity; PCG iterates against scipy's cg with the same
preconditioner; exact solutions of tiny systems against a dense solve.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

from .setup import Hierarchy


def vcycle(h: Hierarchy, f: np.ndarray, level: int = 0) -> np.ndarray:
    lev = h.levels[level]
    if lev.is_coarsest:
        return sla.cho_solve(lev.chol, f)
    x = lev.M @ f
    for _ in range(h.params.npre - 1):
        x = x + lev.M @ (f - lev.A @ x)
    r = f - lev.A @ x
    xc = vcycle(h, lev.R @ r, level + 1)
    x = x + lev.P @ xc
    for _ in range(h.params.npost):
        x = x + lev.Mt @ (f - lev.A @ x)
    return x


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    breakdown: bool
    history: List[float]          # ||r_k|| / ||b|| (recursive residual)
    rel_true_residual: float
    restarts: int


def true_residual_norm(A, b, x) -> float:
    """||b - A x|| / ||b|| in FP64."""
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return float(np.linalg.norm(A @ x))
    return float(np.linalg.norm(b - A @ x) / bn)


def pcg(A, b: np.ndarray, precond: Optional[Callable[[np.ndarray], np.ndarray]] = None,
        tol: float = 1e-8, maxiter: int = 1000, x0: Optional[np.ndarray] = None,
        flexible: bool = False, max_restarts: int = 2) -> SolveResult:
    b = np.asarray(b, dtype=np.float64)
    if precond is None:
        precond = lambda v: v.copy()  # noqa: E731
    bnorm = float(np.linalg.norm(b))
    n = b.shape[0]
    if bnorm == 0.0:
        return SolveResult(np.zeros(n), 0, True, False, [0.0], 0.0, 0)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    history = [float(np.linalg.norm(r)) / bnorm]
    restarts = 0
    it = 0
    if history[-1] <= tol:
        return SolveResult(x, 0, True, False, history, history[-1], 0)
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    converged = breakdown = False
    while it < maxiter:
        q = A @ p
        pq = float(p @ q)
        if not pq > 0.0:
            breakdown = True
            break
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = float(np.linalg.norm(r))
        history.append(rn / bnorm)
        if rn <= tol * bnorm:
            rt = b - A @ x
            if float(np.linalg.norm(rt)) <= tol * bnorm:
                converged = True
                break
            if restarts >= max_restarts:
                break
            restarts += 1
            r = rt
            z = precond(r)
            p = z.copy()
            rz = float(r @ z)
            continue
        z_new = precond(r)
        rz_new = float(r @ z_new)
        if flexible:
            beta = float(r @ (z_new - z)) / rz
        else:
            beta = rz_new / rz
        rz = rz_new
        z = z_new
        p = z + beta * p
    return SolveResult(x, it, converged, breakdown, history,
                       true_residual_norm(A, b, x), restarts)


def amg_pcg(h: Hierarchy, b: np.ndarray, tol: float = 1e-8, maxiter: int = 1000,
            x0=None, flexible: bool = False) -> SolveResult:
    """CG on the finest matrix of ``h`` preconditioned by one V-cycle."""
    A = h.levels[0].A
    return pcg(A, b, lambda r: vcycle(h, r), tol=tol, maxiter=maxiter, x0=x0,
               flexible=flexible)
