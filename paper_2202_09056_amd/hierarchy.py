"""Host-side view of the library's setup (Algorithm 1): build a hierarchy on
the CPU through the C ABI and copy its levels back for inspection."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _capi


def make_params(**kw) -> _capi.AmgParams:
    lib = _capi.load()
    prm = _capi.AmgParams()
    lib.amg_default_params(C.byref(prm))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = _capi.PRECISIONS[v]
        if k == "krylov" and isinstance(v, str):
            v = _capi.KRYLOV[v]
        if k == "smoother" and isinstance(v, str):
            v = _capi.SMOOTHERS[v]
        if k == "setup_path" and isinstance(v, str):
            v = _capi.SETUP_PATHS[v]
        if not hasattr(prm, k):
            raise KeyError(k)
        setattr(prm, k, v)
    return prm


class _HostBsr:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, row_ptr, col, val):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64).reshape(-1)
        nb = self.row_ptr.shape[0] - 1
        self.c = _capi.AmgBsr3(nb, self.col.shape[0], self.row_ptr.ctypes.data,
                               self.col.ctypes.data, self.val.ctypes.data)


class HostHierarchy:
    """The library's host setup (Algorithm 1).  With device_stream (a torch
    stream, or True for the null stream) the numeric phase of the Galerkin
    products runs on the GPU (amg_hierarchy_build_device)."""

    def __init__(self, row_ptr, col, val, coords, device_stream=None, **params):
        self.lib = _capi.load()
        self._A = _HostBsr(row_ptr, col, val)
        self._coords = np.ascontiguousarray(coords, dtype=np.float64)
        prm = make_params(**params)
        h = C.c_void_p()
        if device_stream is None:
            _capi.check(self.lib, self.lib.amg_hierarchy_build(
                C.byref(self._A.c), self._coords.ctypes.data, C.byref(prm), C.byref(h)))
        else:
            sp = None if device_stream is True else C.c_void_p(device_stream.cuda_stream)
            _capi.check(self.lib, self.lib.amg_hierarchy_build_device(
                C.byref(self._A.c), self._coords.ctypes.data, C.byref(prm), sp, C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.lib.amg_hierarchy_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> _capi.AmgStats:
        st = _capi.AmgStats()
        _capi.check(self.lib, self.lib.amg_hierarchy_stats(self.h, C.byref(st)))
        return st

    @property
    def levels(self) -> int:
        return self.stats().levels

    def _shape(self, level, which):
        r, c, n = C.c_int32(), C.c_int32(), C.c_int64()
        _capi.check(self.lib, self.lib.amg_hierarchy_level_shape(
            self.h, level, which, C.byref(r), C.byref(c), C.byref(n)))
        return r.value, c.value, n.value

    def bsr(self, level: int, which: str):
        """('A'|'P'|'R'|'AM'|'G'|'ILU_L'|'ILU_U') -> (row_ptr, col, val[nnzb,3,3], (rows, cols)).
        AM and G are the operators of the fused sweeps of levels below the
        first (empty where a level has none); ILU_L and ILU_U the block ILU(0)
        factors of a level with that smoother (L without its unit diagonal, U
        with its diagonal blocks)."""
        k = {"A": 0, "P": 1, "R": 2, "AM": 9, "G": 10, "ILU_L": 12, "ILU_U": 13}[which]
        rows, cols, nnzb = self._shape(level, k)
        rp = np.zeros(rows + 1, dtype=np.int32)
        col = np.zeros(nnzb, dtype=np.int32)
        val = np.zeros((nnzb, 3, 3), dtype=np.float64)
        _capi.check(self.lib, self.lib.amg_hierarchy_export(
            self.h, level, k, rp.ctypes.data, col.ctypes.data, val.ctypes.data))
        return rp, col, val, (rows, cols)

    def scipy(self, level: int, which: str):
        import scipy.sparse as sp
        rp, col, val, (rows, cols) = self.bsr(level, which)
        return sp.bsr_matrix((val, col, rp), shape=(3 * rows, 3 * cols)).tocsr()

    def smoother_blocks(self, level: int, post: bool = False) -> np.ndarray:
        """Pre-sweep smoother blocks (nb, 3, 3) of a level, or the post-sweep
        blocks (the transposes for SPAI-0)."""
        which = 8 if post else 3
        rows, _, n = self._shape(level, which)
        out = np.zeros((rows, 3, 3))
        if n:
            _capi.check(self.lib, self.lib.amg_hierarchy_export(
                self.h, level, which, None, None, out.ctypes.data))
        return out

    def ilu_colours(self, level: int) -> Optional[np.ndarray]:
        """Colour of each block row of a level with the ILU(0) smoother (None elsewhere)."""
        rows, _, n = self._shape(level, 11)
        if n == 0:
            return None
        out = np.zeros(n)
        _capi.check(self.lib, self.lib.amg_hierarchy_export(self.h, level, 11, None, None, out.ctypes.data))
        return out.astype(np.int64)

    def aggregates(self, level: int) -> Optional[np.ndarray]:
        rows, n_agg, n = self._shape(level, 4)
        if n == 0:
            return None
        out = np.zeros(n)
        _capi.check(self.lib, self.lib.amg_hierarchy_export(
            self.h, level, 4, None, None, out.ctypes.data))
        return out.astype(np.int64)

    def coarse_inverse(self) -> np.ndarray:
        n, _, _ = self._shape(0, 5)
        out = np.zeros((n, n))
        _capi.check(self.lib, self.lib.amg_hierarchy_export(
            self.h, 0, 5, None, None, out.ctypes.data))
        return out

    def learned_inputs(self):
        """(features (nb, 90), Cholesky factors (nb, 6)) of the learned
        smoother, or None when the hierarchy was built without them."""
        rows, per, n = self._shape(0, 6)
        if n == 0:
            return None
        phi = np.zeros(n)
        _capi.check(self.lib, self.lib.amg_hierarchy_export(self.h, 0, 6, None, None, phi.ctypes.data))
        rows7, _, n7 = self._shape(0, 7)
        L = np.zeros(n7)
        _capi.check(self.lib, self.lib.amg_hierarchy_export(self.h, 0, 7, None, None, L.ctypes.data))
        return phi.reshape(rows, per), L.reshape(rows7, 6)
