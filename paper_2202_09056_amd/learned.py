"""Training driver of the learned level-1 smoother blocks.

The network, the blocks it produces, the loss and the optimizer are defined
next to ``amg_smoother_set_weights`` in include/saamg.h; every numerical step
(inference, the loss and its gradient, Adam, the training errors) runs in the
library's HIP kernels.  This module only draws the seeded random numbers
(initial weights, initial errors), loops over the steps and saves or loads the
weights as a versioned ``.npz`` file.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional, Sequence

import numpy as np

from . import _capi
from .solver import Solver

WEIGHTS_VERSION = 1
N_PARAMS = _capi.MLP_PARAMS
LAYOUT = "W1[90][64] b1[64] W2[64][64] b2[64] W3[64][6] b3[6]"


def init_weights(rng: np.random.Generator) -> np.ndarray:
    """He-normal hidden layers, zero output layer (the network starts as block
    Jacobi)."""
    theta = np.zeros(N_PARAMS, dtype=np.float32)
    theta[0:5760] = rng.standard_normal(5760) * np.sqrt(2.0 / 90)
    theta[5824:9920] = rng.standard_normal(4096) * np.sqrt(2.0 / 64)
    return theta


@dataclasses.dataclass
class TrainConfig:
    steps: int = 200
    batch: int = 4            # errors per problem and step
    pool: int = 16            # errors kept per problem, redrawn every `refresh` steps
    refresh: int = 50
    cycles: int = 2           # stationary V-cycle steps applied to the random errors
    lr: float = 1e-3
    lr_late: float = 3e-4     # after late_frac of the steps
    late_frac: float = 0.7
    seed: int = 4
    eps_strong: float = 0.08
    coarse_enough: int = 500  # small training meshes still get two levels


@dataclasses.dataclass
class TrainResult:
    theta: np.ndarray
    losses: List[float]
    seconds: float


def free_mask(row_ptr) -> np.ndarray:
    """1 for the unknowns of nodes with off-diagonal blocks, 0 for nodes whose
    row holds only the diagonal block (eliminated Dirichlet nodes)."""
    lens = np.diff(np.asarray(row_ptr, dtype=np.int64))
    return np.repeat(lens > 1, 3).astype(np.float64)


def train_smoother(problems: Sequence, cfg: Optional[TrainConfig] = None, stream=None,
                   log=None) -> TrainResult:
    """Train on ``problems`` (tuples (row_ptr, col, val, coords)); returns the
    float32 parameter vector and the loss history."""
    import torch
    cfg = cfg or TrainConfig()
    rng = np.random.default_rng(cfg.seed)
    solvers = [Solver(*p, stream=stream, smoother="learned", eps_strong=cfg.eps_strong,
                      coarse_enough=cfg.coarse_enough) for p in problems]
    masks = [torch.from_numpy(free_mask(p[0])).cuda() for p in problems]
    try:
        dev = torch.device("cuda")
        theta = torch.from_numpy(init_weights(rng)).to(dev)
        m = torch.zeros_like(theta)
        v = torch.zeros_like(theta)
        grad = torch.zeros_like(theta)

        def draw():
            # errors of the block-Jacobi method (the loss installs S(theta))
            pools = []
            for s, mask in zip(solvers, masks):
                s.set_smoother_weights(None)
                E = torch.from_numpy(rng.standard_normal((cfg.pool, s.n))).to(dev) * mask
                pools.append(s.training_errors(E.contiguous(), cfg.cycles))
            return pools

        t0 = time.perf_counter()
        pools = draw()
        losses = []
        for t in range(1, cfg.steps + 1):
            if t > 1 and (t - 1) % cfg.refresh == 0:
                pools = draw()
            off = ((t - 1) * cfg.batch) % cfg.pool
            total = 0.0
            for i, (s, E) in enumerate(zip(solvers, pools)):
                total += s.mlp_loss_grad(theta, E[off:off + cfg.batch], grad,
                                         scale=1.0 / len(solvers), accumulate=i > 0)
            lr = cfg.lr if t <= cfg.late_frac * cfg.steps else cfg.lr_late
            solvers[0].mlp_adam(theta, grad, m, v, t, lr)
            losses.append(total / len(solvers))
            if log and (t == 1 or t % 25 == 0):
                log(f"step {t}: loss {losses[-1]:.4f}")
        torch.cuda.synchronize()
        return TrainResult(theta.cpu().numpy(), losses, time.perf_counter() - t0)
    finally:
        for s in solvers:
            s.close()


def save_weights(path: str, theta: np.ndarray, **meta) -> None:
    theta = np.asarray(theta, dtype=np.float32)
    if theta.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    extra = {k: np.asarray(v) for k, v in meta.items()}
    np.savez(path, version=np.int32(WEIGHTS_VERSION), layout=np.array(LAYOUT), theta=theta, **extra)


def load_weights(path: str) -> np.ndarray:
    """Parameters from a file written by save_weights; ValueError if the file
    is not one (wrong version, layout or size, non-finite values)."""
    try:
        with np.load(path, allow_pickle=False) as z:
            version = int(z["version"])
            layout = str(z["layout"])
            theta = np.array(z["theta"], dtype=np.float32)
    except (OSError, KeyError, ValueError) as e:
        raise ValueError(f"{path}: not a smoother weights file ({e})") from e
    if version != WEIGHTS_VERSION or layout != LAYOUT:
        raise ValueError(f"{path}: weights version {version} / layout {layout!r} not supported")
    if theta.shape != (N_PARAMS,) or not np.isfinite(theta).all():
        raise ValueError(f"{path}: expected {N_PARAMS} finite parameters")
    return theta
