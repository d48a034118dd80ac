"""Block <-> scalar CSR conversion (oracle side; test infrastructure only).

Section 2 defines the block-valued CSR format by a worked 6x6 example with
2x2 blocks: ``ptr`` indexes block rows, ``col`` holds block column indices and
``val`` holds one small dense block per entry.  A block is stored whenever any
scalar entry inside it is structurally present.

Pinned by the exact arrays of that worked example (tests/golden) and by a
round trip through scipy's bsr_matrix.
"""
import numpy as np
import scipy.sparse as sp


def csr_to_bsr(ptr, col, val, n, bs):
    """Scalar CSR (n x n) -> block CSR with bs x bs blocks.

    Returns (bptr, bcol, bval) with bval of shape [nnzb, bs, bs]; block
    columns are sorted within each block row.
    """
    ptr = np.asarray(ptr); col = np.asarray(col); val = np.asarray(val, dtype=np.float64)
    assert n % bs == 0
    nb = n // bs
    bptr = [0]
    bcol = []
    bval = []
    for I in range(nb):
        blocks = {}
        for r in range(bs):
            i = I * bs + r
            for k in range(ptr[i], ptr[i + 1]):
                J = int(col[k]) // bs
                if J not in blocks:
                    blocks[J] = np.zeros((bs, bs))
                blocks[J][r, int(col[k]) % bs] += val[k]
        for J in sorted(blocks):
            bcol.append(J)
            bval.append(blocks[J])
        bptr.append(len(bcol))
    return (np.array(bptr, dtype=np.int64), np.array(bcol, dtype=np.int64),
            np.array(bval).reshape(-1, bs, bs))


def bsr_to_csr(bptr, bcol, bval, keep_zeros=True):
    """Block CSR -> scalar CSR; scalar entries keep block order within a row."""
    bptr = np.asarray(bptr); bcol = np.asarray(bcol); bval = np.asarray(bval)
    bs = bval.shape[1]
    nb = len(bptr) - 1
    ptr = [0]
    col = []
    val = []
    for I in range(nb):
        for r in range(bs):
            for k in range(bptr[I], bptr[I + 1]):
                for c in range(bs):
                    v = bval[k, r, c]
                    if keep_zeros or v != 0.0:
                        col.append(int(bcol[k]) * bs + c)
                        val.append(float(v))
            ptr.append(len(col))
    return np.array(ptr, dtype=np.int64), np.array(col, dtype=np.int64), np.array(val)


def to_scipy_bsr(A: sp.spmatrix, bs: int = 3) -> sp.bsr_matrix:
    """A scipy block view of a scalar matrix (used for the oracle's own block form)."""
    return sp.bsr_matrix(A, blocksize=(bs, bs))
