"""Device solver handle: thin wrapper over the C ABI (argument marshalling only).

Vectors are PyTorch tensors on the GPU (float64, contiguous); PyTorch supplies
device memory and the stream, every step of the solve runs in the library's
HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _capi
from .hierarchy import HostHierarchy, _HostBsr, make_params


def _torch():
    import torch
    return torch


def _dptr(t, n: Optional[int] = None) -> int:
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} entries, got {t.numel()}")
    return t.data_ptr()


def _fptr(t, n: Optional[int] = None) -> int:
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("expected a contiguous float32 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} entries, got {t.numel()}")
    return t.data_ptr()


class Solver:
    """SA-AMG preconditioned CG on one GPU.

    Build from a host BSR3 matrix and node coordinates (``Solver(row_ptr, col,
    val, coords, **params)``) or from an existing :class:`HostHierarchy`
    (``Solver.from_hierarchy(h, **params)``).
    """

    def __init__(self, row_ptr=None, col=None, val=None, coords=None, stream=None,
                 _hier: Optional[HostHierarchy] = None, **params):
        torch = _torch()
        self.lib = _capi.load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.prm = make_params(**params)
        ctx = C.c_void_p()
        sptr = C.c_void_p(stream.cuda_stream)
        if _hier is not None:
            _capi.check(self.lib, self.lib.amg_upload(_hier.h, C.byref(self.prm), sptr, C.byref(ctx)))
        else:
            A = _HostBsr(row_ptr, col, val)
            xyz = np.ascontiguousarray(coords, dtype=np.float64)
            _capi.check(self.lib, self.lib.amg_setup(C.byref(A.c), xyz.ctypes.data, C.byref(self.prm),
                                                     sptr, C.byref(ctx)))
        self.ctx = ctx
        self.n = 3 * self.stats().nb[0]

    @classmethod
    def from_hierarchy(cls, hier: HostHierarchy, stream=None, **params):
        return cls(stream=stream, _hier=hier, **params)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.amg_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> _capi.AmgStats:
        st = _capi.AmgStats()
        _capi.check(self.lib, self.lib.amg_stats(self.ctx, C.byref(st)))
        return st

    def solve(self, b, x=None, tol: float = 1e-8, raise_on_error: bool = True):
        """Solve A x = b; returns (x, info, status)."""
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        info = _capi.AmgSolveInfo()
        s = self.lib.amg_solve(self.ctx, C.c_void_p(_dptr(b, self.n)), C.c_void_p(_dptr(x, self.n)),
                               C.c_double(tol), C.byref(info))
        if raise_on_error:
            _capi.check(self.lib, s)
        return x, info, s

    def solve_multi(self, B, X=None, tol: float = 1e-8, raise_on_error: bool = True):
        """Solve A X = B for B of shape (n, k), k <= 32 (row-major); returns
        (X, [info per column], status)."""
        torch = _torch()
        if B.dim() != 2 or B.shape[0] != self.n or not 1 <= B.shape[1] <= 32:
            raise ValueError("B must have shape (n, k) with 1 <= k <= 32")
        k = int(B.shape[1])
        if X is None:
            X = torch.zeros_like(B)
        if tuple(X.shape) != tuple(B.shape):
            raise ValueError("X must have the shape of B")
        infos = (_capi.AmgSolveInfo * k)()
        s = self.lib.amg_solve_multi(self.ctx, k, C.c_void_p(_dptr(B, self.n * k)),
                                     C.c_void_p(_dptr(X, self.n * k)), C.c_double(tol), infos)
        if raise_on_error:
            _capi.check(self.lib, s)
        return X, list(infos), s

    def vcycle(self, r, z=None):
        torch = _torch()
        if z is None:
            z = torch.empty_like(r)
        _capi.check(self.lib, self.lib.amg_vcycle(self.ctx, C.c_void_p(_dptr(r, self.n)),
                                                  C.c_void_p(_dptr(z, self.n))))
        return z

    def vcycle_multi(self, R, Z=None):
        """Z = V(R) column by column for R of shape (n, k), k <= 32, in one
        multi-column V-cycle."""
        torch = _torch()
        if R.dim() != 2 or R.shape[0] != self.n or not 1 <= R.shape[1] <= 32:
            raise ValueError("R must have shape (n, k) with 1 <= k <= 32")
        if Z is None:
            Z = torch.empty_like(R)
        k = int(R.shape[1])
        _capi.check(self.lib, self.lib.amg_vcycle_multi(self.ctx, k, C.c_void_p(_dptr(R, self.n * k)),
                                                        C.c_void_p(_dptr(Z, self.n * k))))
        return Z

    def debug_apply(self, level: int, op: int, inp, out, in2=None):
        st = self.stats()
        if op == 5:
            n_in = n_out = st.n_coarse
        else:
            if not 0 <= level < st.levels - 1:
                raise ValueError("level has no sparse operators")
            n_f, n_c = 3 * st.nb[level], 3 * st.nb[level + 1]
            n_in, n_out = {0: (n_f, n_f), 1: (n_f, n_c), 2: (n_c, n_f), 3: (n_f, n_f),
                           4: (n_f, n_f), 6: (n_f, n_f), 11: (n_f, n_f), 12: (n_c, n_f)}[op]
        p2 = C.c_void_p(_dptr(in2, n_out)) if in2 is not None else None
        _capi.check(self.lib, self.lib.amg_debug_apply(self.ctx, level, op, C.c_void_p(_dptr(inp, n_in)),
                                                       p2, C.c_void_p(_dptr(out, n_out))))
        return out

    def true_residual(self, b, x) -> float:
        rel = C.c_double()
        _capi.check(self.lib, self.lib.amg_true_residual(self.ctx, C.c_void_p(_dptr(b, self.n)),
                                                         C.c_void_p(_dptr(x, self.n)), C.byref(rel)))
        return rel.value

    def true_residual_noalloc(self, b, x, r, norms, sync: bool = True):
        """r = b - A x and norms = (||b||^2, ||r||^2) with the library's static
        scratch (no device allocation); returns ||r||/||b|| if sync, else None
        (only enqueued on the context stream)."""
        rel = C.c_double()
        _capi.check(self.lib, self.lib.amg_true_residual_noalloc(
            self.ctx, C.c_void_p(_dptr(b, self.n)), C.c_void_p(_dptr(x, self.n)), C.c_void_p(_dptr(r, self.n)),
            C.c_void_p(_dptr(norms, 2)), C.byref(rel) if sync else None))
        return rel.value if sync else None

    def time_op(self, level: int, op: int, reps: int = 20):
        """(mean ms per launch, algorithmic bytes per launch) of one kernel."""
        ms, nbytes = C.c_double(), C.c_double()
        _capi.check(self.lib, self.lib.amg_time_op(self.ctx, level, op, reps, C.byref(ms),
                                                   C.byref(nbytes)))
        return ms.value, nbytes.value

    # ---- learned level-1 smoother blocks (smoother="learned" at setup) ----

    def set_smoother_weights(self, theta=None, check: bool = True) -> int:
        """Install the learned blocks of ``theta`` (float32 or bfloat16 CUDA
        tensor of MLP_PARAMS entries) or, with None, restore block Jacobi.
        Returns the number of nodes that kept their block-Jacobi block."""
        torch = _torch()
        nbad = C.c_int32(0)
        if theta is None:
            ptr, nbytes, dtype = None, 0, _capi.PRECISIONS["fp32"]
        else:
            if not isinstance(theta, torch.Tensor) or not theta.is_cuda or not theta.is_contiguous():
                raise TypeError("theta must be a contiguous CUDA tensor")
            if theta.numel() != _capi.MLP_PARAMS:
                raise ValueError(f"theta needs {_capi.MLP_PARAMS} entries")
            if theta.dtype == torch.float32:
                dtype = _capi.PRECISIONS["fp32"]
            elif theta.dtype == torch.bfloat16:
                dtype = _capi.PRECISIONS["bf16"]
            else:
                raise TypeError("theta must be float32 or bfloat16")
            ptr, nbytes = C.c_void_p(theta.data_ptr()), theta.numel() * theta.element_size()
        _capi.check(self.lib, self.lib.amg_smoother_set_weights(self.ctx, ptr, nbytes, dtype, int(check),
                                                                C.byref(nbad)))
        return nbad.value

    def mlp_loss_grad(self, theta, E, grad, scale: float = 1.0, accumulate: bool = False) -> float:
        """Two-grid energy loss of ``theta`` over the columns of E (float64
        CUDA tensor of shape (k, n)); scale * gradient into ``grad``."""
        if E.dim() != 2 or E.shape[1] != self.n:
            raise ValueError("E must have shape (k, n)")
        loss = C.c_double()
        _capi.check(self.lib, self.lib.amg_mlp_loss_grad(
            self.ctx, C.c_void_p(_fptr(theta, _capi.MLP_PARAMS)), C.c_void_p(_dptr(E, E.numel())),
            int(E.shape[0]), C.c_float(scale), int(accumulate), C.byref(loss),
            C.c_void_p(_fptr(grad, _capi.MLP_PARAMS))))
        return loss.value

    def mlp_adam(self, theta, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8):
        n = theta.numel()
        _capi.check(self.lib, self.lib.amg_mlp_adam(
            self.ctx, C.c_void_p(_fptr(theta, n)), C.c_void_p(_fptr(grad, n)), C.c_void_p(_fptr(m, n)),
            C.c_void_p(_fptr(v, n)), n, int(step), C.c_float(lr), C.c_float(beta1), C.c_float(beta2),
            C.c_float(eps)))

    def training_errors(self, E, cycles: int):
        """In place: every row e of E (shape (k, n)) becomes e - V(A e), ``cycles`` times."""
        if E.dim() != 2 or E.shape[1] != self.n:
            raise ValueError("E must have shape (k, n)")
        _capi.check(self.lib, self.lib.amg_training_errors(self.ctx, C.c_void_p(_dptr(E, E.numel())),
                                                           int(E.shape[0]), int(cycles)))
        return E


class BatchSolver:
    """Many independent problems solved together (one launch per V-cycle step
    for the whole batch).  problems: list of (row_ptr, col, val, coords)."""

    def __init__(self, problems, stream=None, **params):
        torch = _torch()
        self.lib = _capi.load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.prm = make_params(**params)
        self._mats = [_HostBsr(rp, col, val) for (rp, col, val, _) in problems]
        self._xyz = [np.ascontiguousarray(c, dtype=np.float64) for (_, _, _, c) in problems]
        self.np = len(problems)
        self.sizes = [3 * (len(rp) - 1) for (rp, _, _, _) in problems]
        arr = (_capi.AmgBsr3 * self.np)(*[m.c for m in self._mats])
        ptrs = (C.c_void_p * self.np)(*[x.ctypes.data for x in self._xyz])
        h = C.c_void_p()
        _capi.check(self.lib, self.lib.amg_setup_batch(self.np, arr, ptrs, C.byref(self.prm),
                                                       C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.amg_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vcycle(self, rs, zs=None):
        """One batched V-cycle: zs[p] = V_p(rs[p]) for every problem."""
        torch = _torch()
        if len(rs) != self.np:
            raise ValueError("one vector per problem")
        if zs is None:
            zs = [torch.empty_like(r) for r in rs]
        rp = (C.c_void_p * self.np)(*[_dptr(r, n) for r, n in zip(rs, self.sizes)])
        zp = (C.c_void_p * self.np)(*[_dptr(z, n) for z, n in zip(zs, self.sizes)])
        _capi.check(self.lib, self.lib.amg_vcycle_batch(self.h, rp, zp))
        return zs

    def solve(self, bs, xs=None, tol: float = 1e-8, raise_on_error: bool = True):
        """bs: list of device float64 vectors; returns (xs, infos, status)."""
        torch = _torch()
        if len(bs) != self.np:
            raise ValueError("one right-hand side per problem")
        if xs is None:
            xs = [torch.zeros_like(b) for b in bs]
        bp = (C.c_void_p * self.np)(*[_dptr(b, n) for b, n in zip(bs, self.sizes)])
        xp = (C.c_void_p * self.np)(*[_dptr(x, n) for x, n in zip(xs, self.sizes)])
        infos = (_capi.AmgSolveInfo * self.np)()
        s = self.lib.amg_solve_batch(self.h, bp, xp, C.c_double(tol), infos)
        if raise_on_error:
            _capi.check(self.lib, s)
        return xs, list(infos), s
