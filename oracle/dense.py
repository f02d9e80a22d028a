"""Tiny grids only: the interior-node operator L_h as a dense matrix.

Eliminating the interface unknowns with the flux rows of the collocation
system (their right-hand side is always zero) leaves
    Ktil = K_ii - K_iG K_GG^{-1} K_Gi
on the interior nodes, and the discrete first-order operator
    L_h = [[0, I], [Ktil, 0]]
whose resolvents are exactly the solves of ``collocation``.  Hence the step
sum_m b_m (tau L_h - alpha_m)^{-1} equals R(tau L_h) = V R(tau Lambda) V^{-1}
for L_h = V Lambda V^{-1} (section 1.2, eqs. def_RM and error-in-exp), and
the true propagator is V e^{tau Lambda} V^{-1}.

Parity role: brute-force check of the oracle's solves and pole sum on tiny
grids (eigendecomposition and dense solves, independent of the sparse LU).
"""
from __future__ import annotations

import numpy as np

from .rational import R_eval


def interior_operator(K, n_int: int) -> np.ndarray:
    A = K.toarray()
    Kii, KiG = A[:n_int, :n_int], A[:n_int, n_int:]
    KGi, KGG = A[n_int:, :n_int], A[n_int:, n_int:]
    if KGG.shape[0] == 0:
        return Kii
    return Kii - KiG @ np.linalg.solve(KGG, KGi)


def first_order_operator(Ktil: np.ndarray) -> np.ndarray:
    n = Ktil.shape[0]
    L = np.zeros((2 * n, 2 * n))
    L[:n, n:] = np.eye(n)
    L[n:, :n] = Ktil
    return L


def dense_resolvent(L: np.ndarray, tau: float, alpha: complex, u0, v0):
    """(tau L - alpha)^{-1} (u0, v0) by a dense solve of the 2n system."""
    n = L.shape[0] // 2
    rhs = np.concatenate([u0, v0]).astype(np.complex128)
    y = np.linalg.solve(tau * L - alpha * np.eye(2 * n), rhs)
    return y[:n], y[n:]


def eig_step(L: np.ndarray, tau: float, alpha, b, u0, v0, n_steps: int = 1):
    """R(tau L)^n (u0, v0) through the eigendecomposition of L."""
    lam, V = np.linalg.eig(L)
    w = np.linalg.solve(V, np.concatenate([u0, v0]).astype(np.complex128))
    w = w * R_eval(alpha, b, tau * lam) ** n_steps
    y = V @ w
    n = L.shape[0] // 2
    return y[:n], y[n:]


def eig_exact(L: np.ndarray, t: float, u0, v0):
    """e^{t L} (u0, v0) through the eigendecomposition of L."""
    lam, V = np.linalg.eig(L)
    w = np.linalg.solve(V, np.concatenate([u0, v0]).astype(np.complex128))
    y = V @ (w * np.exp(t * lam))
    n = L.shape[0] // 2
    return y[:n], y[n:]
