"""Pins for the oracle's block <-> scalar CSR conversion (CPU only).

The exact arrays of the paper's worked example (Section 2, 6x6 matrix with
2x2 blocks) are stored in tests/golden/paper_bsr_example.json.
"""
import json
import os

import numpy as np
import scipy.sparse as sp

import meshgen
from oracle import formats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_bsr_example.json")


def _load():
    with open(GOLDEN) as f:
        return json.load(f)


def test_paper_example_csr_to_bsr_exact():
    g = _load()
    c = g["csr"]
    bptr, bcol, bval = formats.csr_to_bsr(c["ptr"], c["col"], c["val"], 6, 2)
    assert bptr.tolist() == g["bsr"]["ptr"]
    assert bcol.tolist() == g["bsr"]["col"]
    assert np.array_equal(bval, np.array(g["bsr"]["val"]))


def test_paper_example_bsr_to_csr_exact():
    g = _load()
    b = g["bsr"]
    ptr, col, val = formats.bsr_to_csr(b["ptr"], b["col"], np.array(b["val"]), keep_zeros=False)
    assert ptr.tolist() == g["csr"]["ptr"]
    assert col.tolist() == g["csr"]["col"]
    assert np.array_equal(val, np.array(g["csr"]["val"]))
    # and the CSR arrays describe the printed dense matrix
    dense = sp.csr_matrix((val, col, ptr), shape=(6, 6)).toarray()
    assert np.array_equal(dense, np.array(g["dense"]))


def test_paper_example_index_memory_ratios():
    """Block form: half the ptr entries (rows / 2) and a quarter of the col
    entries (2x2 blocks), as stated for the example."""
    g = _load()
    assert len(g["csr"]["ptr"]) - 1 == 2 * (len(g["bsr"]["ptr"]) - 1)
    assert len(g["csr"]["col"]) == 4 * len(g["bsr"]["col"])


def test_bs3_round_trip_against_scipy():
    p = meshgen.cube_c1(3)
    A = p.csr()
    bptr, bcol, bval = formats.csr_to_bsr(A.indptr, A.indices, A.data, A.shape[0], 3)
    ref = sp.bsr_matrix(A, blocksize=(3, 3))
    ref.sort_indices()
    assert np.array_equal(bptr, ref.indptr) and np.array_equal(bcol, ref.indices)
    assert np.array_equal(bval, ref.data)
    ptr, col, val = formats.bsr_to_csr(bptr, bcol, bval)
    back = sp.csr_matrix((val, col, ptr), shape=A.shape)
    assert abs(back - A).max() == 0.0
    # 3x3 blocks: ptr shrinks by 3, col by 9 when every block is full
    assert len(bptr) - 1 == (len(A.indptr) - 1) // 3
