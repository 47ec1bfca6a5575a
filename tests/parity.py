"""Comparison measures shared by the GPU parity tests.

Every result (one output row of a signal, one image, one sampled set of points) is compared
with its FP64 oracle value by two measures, and both must stay within the stated tolerance:

  * relative L2:  ||y - y_ref||_2 / ||y_ref||_2
  * relative max: max_i |y_i - y_ref_i| / max_i |y_ref_i|      (element by element)

The second catches a single wrong element that the first would average away: at 16384
outputs a relative L2 of 1e-5 still admits one element off by about 1e-3 of the signal's
RMS.  Complex values are compared by modulus.
"""
import numpy as np


def _f(a):
    a = np.asarray(a)
    return a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)


def rows(a, n):
    return _f(a).reshape(n, -1)


def rel_l2(got, want):
    """Per-row relative L2 error over the leading axis."""
    g, w = _f(got), _f(want)
    n = g.shape[0] if g.ndim > 1 else 1
    g, w = g.reshape(n, -1), w.reshape(n, -1)
    return np.linalg.norm(g - w, axis=1) / np.maximum(np.linalg.norm(w, axis=1), 1e-300)


def rel_max(got, want):
    """Per-row element-wise error, max |y - y_ref| / max |y_ref|, over the leading axis."""
    g, w = _f(got), _f(want)
    n = g.shape[0] if g.ndim > 1 else 1
    g, w = g.reshape(n, -1), w.reshape(n, -1)
    return np.abs(g - w).max(axis=1, initial=0.0) / np.maximum(np.abs(w).max(axis=1, initial=0.0), 1e-300)


def check_rows(got, want, tol, what=""):
    """Assert both measures <= tol for every row of got/want (leading axis); returns (l2, mx)."""
    l2, mx = rel_l2(got, want), rel_max(got, want)
    assert l2.max() <= tol and mx.max() <= tol, (
        f"{what} rel L2 max {l2.max():.3e} (median {np.median(l2):.3e}), "
        f"rel max-abs max {mx.max():.3e} (median {np.median(mx):.3e}), tol {tol:.0e}")
    return l2, mx


def check(got, want, tol, what=""):
    """Assert both measures <= tol with got/want taken as one result; returns (l2, mx)."""
    g, w = _f(got).reshape(1, -1), _f(want).reshape(1, -1)
    l2, mx = check_rows(g, w, tol, what)
    return float(l2[0]), float(mx[0])


def worst(got, want):
    """max(relative L2, relative max-abs) with got/want taken as one result."""
    g, w = _f(got).reshape(1, -1), _f(want).reshape(1, -1)
    return float(max(rel_l2(g, w)[0], rel_max(g, w)[0]))


def worst_rows(got, want):
    """max over the rows of the leading axis of max(relative L2, relative max-abs)."""
    return float(max(rel_l2(got, want).max(), rel_max(got, want).max()))
