"""Chebyshev-Lobatto nodes and the spectral differentiation matrix.

Section 2.2 of the paper tabulates functions on a p x p tensor grid of
Chebyshev nodes per element and replaces derivatives by spectral
differentiation on that grid.  The differentiation matrix below is the
classical one for the points x_k = cos(k pi / N), N = p - 1 (e.g. Trefethen,
"Spectral Methods in MATLAB", ch. 6), reordered so that nodes ascend.

Pinned by: exactness on polynomials of degree <= p-1 (tests).
"""
from __future__ import annotations

import numpy as np


def nodes(p: int) -> np.ndarray:
    """Chebyshev-Lobatto points on [-1, 1] in ascending order."""
    N = p - 1
    return -np.cos(np.pi * np.arange(p) / N)


def diff_matrix(p: int) -> np.ndarray:
    """D with (D f)(x_i) = f'(x_i) for polynomials f of degree <= p-1,
    rows/columns in the ascending node order of ``nodes``."""
    N = p - 1
    k = np.arange(p)
    x = np.cos(np.pi * k / N)                     # descending
    c = np.ones(p)
    c[0] = c[-1] = 2.0
    c = c * (-1.0) ** k
    dx = x[:, None] - x[None, :]
    D = np.outer(c, 1.0 / c) / (dx + np.eye(p))
    D = D - np.diag(D.sum(axis=1))
    # ascending order: x_asc[i] = x[N - i]; d/dx is unchanged by relabelling
    return D[::-1, ::-1].copy()


def unit_nodes(p: int) -> np.ndarray:
    """The same nodes mapped to [0, 1]."""
    return 0.5 * (nodes(p) + 1.0)
