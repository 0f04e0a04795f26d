"""Comparison helpers for the tests (no refinement arithmetic here)."""
import numpy as np


def align_signs(X, Xref):
    """Flip each column of X to the sign of its inner product with Xref;
    eigenvectors are only defined up to sign."""
    X = np.asarray(X)
    s = np.sign(np.sum(X * np.asarray(Xref), axis=0))
    s[s == 0] = 1.0
    return X * s


def max_abs_diff_aligned(X, Xref):
    return float(np.max(np.abs(align_signs(X, Xref) - np.asarray(Xref))))


def sin_theta(X, Xref):
    """Sine of the largest principal angle between span(X) and span(Xref)."""
    qa, _ = np.linalg.qr(np.asarray(X))
    qb, _ = np.linalg.qr(np.asarray(Xref))
    s = np.linalg.svd(qa.T @ qb, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - np.min(s) ** 2)))
