"""Element-wise comparison of a device result with the oracle's.

Every entry is held to |a_i - b_i| <= rtol |b_i| + atol * max_j |b_j|: a
relative bound per entry with an absolute floor at the scale of the whole
vector (entries that cancel to nearly zero carry the rounding of the terms
that produced them, which is of the order of the largest entries).  An
error confined to a few rows, or to the small entries, fails it even when
the vector's norm hardly moves.
"""
import numpy as np


def assert_close(a, b, rtol, atol, what=""):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    assert a.shape == b.shape, (what, a.shape, b.shape)
    assert np.all(np.isfinite(a)), (what, "non-finite entries")
    scale = float(np.abs(b).max()) if b.size else 0.0
    bound = rtol * np.abs(b) + atol * scale
    err = np.abs(a - b)
    bad = err > bound
    if bad.any():
        i = int(np.argmax(err - bound))
        raise AssertionError(f"{what}: {int(bad.sum())} of {a.size} entries out of bound; worst at {i}: "
                             f"got {a[i]!r}, expected {b[i]!r}, |diff| {err[i]:.3e} > {bound[i]:.3e} "
                             f"(rtol {rtol}, atol {atol} x max {scale:.3e})")


def assert_close_rows(y, ref, scale, k, what=""):
    """Products and residuals: |y_i - ref_i| <= k u scale_i per entry with
    u = 2^-53 and scale_i = (|A| |x|)_i (+ |b_i| for a residual b - A x): the
    forward error bound of a dot product of the row's length on both sides
    (k absorbs the row length)."""
    y = np.asarray(y, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    bound = k * 2.0 ** -53 * np.asarray(scale, dtype=np.float64).ravel() + 1e-300
    err = np.abs(y - ref)
    bad = err > bound
    if bad.any():
        i = int(np.argmax(err / bound))
        raise AssertionError(f"{what}: {int(bad.sum())} of {y.size} rows out of bound; worst at {i}: "
                             f"|diff| {err[i]:.3e} > {bound[i]:.3e}")


def assert_close_scaled(y, ref, scale, rel, what=""):
    """|y_i - ref_i| <= rel * scale_i per entry, with scale_i the magnitude of
    the terms that make up entry i (for a product A u: (|A| |u|)_i), so the
    bound follows each row's own rounding scale."""
    y = np.asarray(y, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    bound = rel * np.asarray(scale, dtype=np.float64).ravel() + 1e-300
    err = np.abs(y - ref)
    bad = err > bound
    if bad.any():
        i = int(np.argmax(err / bound))
        raise AssertionError(f"{what}: {int(bad.sum())} of {y.size} entries out of bound; worst at {i}: "
                             f"got {y[i]!r}, expected {ref[i]!r}, |diff| {err[i]:.3e} > {bound[i]:.3e}")
