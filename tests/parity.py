"""Element-wise parity measures shared by the GPU tests.

W (m x r) is compared row by row and H (r x k) column by column: the W half of an MU or
BCD iteration computes row i of W from row i of X H^T and of W alone, and the H half
computes column j of H from column j of W^T X and of H alone, so rounding differences
stay relative to the row (or column) they are made in.  A whole-matrix Frobenius ratio
would let one wrong column of a long H hide behind the others.
"""
import numpy as np

TINY = 1e-300  # a zero row (column) of the reference is compared absolutely


def rows_rel(a, b):
    """max_i ||a_i - b_i|| / ||b_i|| over the rows of two m x r matrices."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    if a.size == 0:
        return 0.0
    a2 = a.reshape(a.shape[0], -1)
    b2 = b.reshape(b.shape[0], -1)
    num = np.linalg.norm(a2 - b2, axis=1)
    den = np.maximum(np.linalg.norm(b2, axis=1), TINY)
    return float(np.max(num / den))


def cols_rel(a, b):
    """max_j ||a[:, j] - b[:, j]|| / ||b[:, j]|| over the columns of two r x k matrices."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    return rows_rel(a.reshape(a.shape[0], -1).T, b.reshape(b.shape[0], -1).T)


def cores_rel(got, ref):
    """Worst element-wise error over the cores of a TT sweep: core l < d is stage l's W
    (rows of (r_{l-1} n_l) x r_l), the last core is the last stage's H (columns of
    r_{d-1} x n_d)."""
    worst = 0.0
    for i, (g, o) in enumerate(zip(got, ref)):
        g = np.asarray(g, dtype=np.float64)
        o = np.asarray(o, dtype=np.float64)
        assert g.shape == o.shape, (i, g.shape, o.shape)
        if i < len(ref) - 1:
            e = rows_rel(g.reshape(-1, o.shape[2]), o.reshape(-1, o.shape[2]))
        else:
            e = cols_rel(g.reshape(o.shape[0], -1), o.reshape(o.shape[0], -1))
        worst = max(worst, e)
    return worst


def entries_rel(a, b):
    """max |a - b| / |b| over all entries (b > 0 everywhere, e.g. a TT reconstruction from
    positive cores)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), TINY)))
