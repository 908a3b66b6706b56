"""Naive O(N^2) discrete sine transform of type I.

Test infrastructure only (see the package docstring).

The transform of Lemma 4 / Corollary 1 (Section 3): for a sequence x_m,
m = 1..N-1, X_k = sum_m x_m sin(pi k m / N), k = 1..N-1 (the paper's
coefficients g_hat carry an extra factor 2/N, which is the inverse scaling:
S S = (N/2) I).  The sine matrix is formed with exact integer argument
reduction (k m mod 2N) and extended precision, then rounded to FP64.
"""
from __future__ import annotations

import functools

import numpy as np


@functools.lru_cache(maxsize=32)
def sine_matrix(N: int) -> np.ndarray:
    k = np.arange(1, N, dtype=np.int64)
    km = np.outer(k, k) % (2 * N)
    return np.sin(np.pi * km.astype(np.longdouble) / N).astype(np.float64)


def dst1(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """X = S x along `axis` (length N-1), summed in extended precision."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[axis] + 1
    S = sine_matrix(N).astype(np.longdouble)
    xm = np.moveaxis(x, axis, -1).astype(np.longdouble)
    out = xm @ S.T
    return np.moveaxis(out.astype(np.float64), -1, axis)
