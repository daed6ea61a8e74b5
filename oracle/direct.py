"""Direct O(N^2) evaluation of the potential sum (test infrastructure only).

Eq. (1), Sec. 2.1: p_i = sum_j G(x_i, y_j) q_j with the single-layer Laplace
kernel G(x, y) = 1 / (4 pi |x - y|) stated with the BIE of Sec. 4. The point
form used here has no element integral for the diagonal, so a pair at
distance 0 (the self term, or exact duplicates) contributes 0.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def kernel_matrix(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """G(x_i, y_j) for all pairs, FP64, with G := 0 where x_i == y_j."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = x[:, None, :] - y[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    with np.errstate(divide="ignore"):
        g = 1.0 / (FOUR_PI * r)
    g[r == 0.0] = 0.0
    return g


def direct(x: np.ndarray, sigma: np.ndarray, targets: np.ndarray | None = None,
           sources: np.ndarray | None = None, chunk: int = 512) -> np.ndarray:
    """Potential at `targets` (default: the source points themselves).

    x:       (N,3) source points y_j.
    sigma:   (N,) or (N,m) source densities q_j.
    targets: optional (M,3) evaluation points x_i; defaults to x.
    Returns (M,) or (M,m) in FP64.
    """
    y = np.asarray(x if sources is None else sources, dtype=np.float64)
    t = y if targets is None else np.asarray(targets, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    out = np.zeros((t.shape[0],) + s.shape[1:], dtype=np.float64)
    for a in range(0, t.shape[0], chunk):
        out[a:a + chunk] = kernel_matrix(t[a:a + chunk], y) @ s
    return out
