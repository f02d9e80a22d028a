"""Rational functions of section 1.2 and section 3, evaluated directly.

* ``R_eval``: R(z) = sum_m b_m / (z - alpha_m), the definition of eq. def_RM.
* ``fit_error`` / ``max_modulus``: the two properties eq. RM_prop1 and
  eq. RM_prop2 ask of R on the imaginary axis, checked on dense grids.
* ``table1_gaussian``: the paper's rational approximation of
  psi_1(x) = (4 pi)^{-1/2} e^{-x^2/4} with the coefficients of Table 1, in
  the form Re sum_j a_j / (ix + mu + ij) of section 3.2.
* ``gaussian_sum_exp``: the Gaussian-sum approximation of section 3.1,
  e^{ix} ~ sum_m c_m psi_h(x + m h) with c_m = (h / psi_h^(xi0)) e^{-i m h},
  xi0 = 1/(2 pi) the frequency of e^{ix} and psi_h^ the Fourier transform
  of psi_h (convention f^(xi) = int f(x) e^{-2 pi i x xi} dx), i.e.
  c_m = e^{h^2} e^{-i m h}; the bound of the appendix applies.

Pinned by: Table 1's printed error (about 7e-13), the Poisson-summation
bound of the appendix, closed-form partial fractions (tests).
"""
from __future__ import annotations

import numpy as np


def R_eval(alpha: np.ndarray, b: np.ndarray, z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.complex128)
    out = np.zeros(z.shape, dtype=np.complex128)
    for a, c in zip(alpha, b):
        out += c / (z - a)
    return out


def fit_error(alpha, b, X: float, n: int = 20001) -> float:
    """max |R(ix) - e^{ix}| over a uniform grid of [-X, X]."""
    x = np.linspace(-X, X, n)
    return float(np.abs(R_eval(alpha, b, 1j * x) - np.exp(1j * x)).max())


def max_modulus(alpha, b, x_max: float = 1e7) -> float:
    """max |R(ix)| over a dense grid of [-400, 400] plus geometric grids
    out to +-x_max (R is proper, so |R(ix)| -> 0 beyond)."""
    x = np.concatenate([np.linspace(-400.0, 400.0, 80001),
                        np.geomspace(400.0, x_max, 4000),
                        -np.geomspace(400.0, x_max, 4000)])
    return float(np.abs(R_eval(alpha, b, 1j * x)).max())


def psi(x, h=1.0):
    return (4 * np.pi) ** -0.5 * np.exp(-x ** 2 / (4 * h * h))


def psi_hat(xi, h=1.0):
    """Fourier transform of psi_h: h exp(-4 pi^2 h^2 xi^2)."""
    return h * np.exp(-4 * np.pi ** 2 * h * h * xi ** 2)


def gaussian_sum_exp(x, M: int, h: float = 1.0):
    """sum_{m=-M}^{M} c_m psi_h(x + m h) with the coefficients above."""
    xi0 = 1.0 / (2 * np.pi)
    out = np.zeros(np.shape(x), dtype=np.complex128)
    for m in range(-M, M + 1):
        cm = (h / psi_hat(xi0, h)) * np.exp(-2j * np.pi * m * h * xi0)
        out += cm * psi(x + m * h, h)
    return out


def gaussian_sum_bound(x, M: int, h: float = 1.0, kmax: int = 50):
    """Right-hand side of the appendix bound for e^{ix}:
    (1/psi_h^(xi0)) (sum_{k!=0} psi_h^(k/h) + sum_{|m|>M} psi_h(x + m h)),
    with the first sum taken at the shifted frequencies k/h + xi0 that the
    Poisson summation of the appendix produces."""
    xi0 = 1.0 / (2 * np.pi)
    ks = np.concatenate([np.arange(-kmax, 0), np.arange(1, kmax + 1)])
    alias = np.sum(psi_hat(ks / h + xi0, h)) / h
    tail = np.zeros(np.shape(x))
    for m in list(range(-M - 200, -M)) + list(range(M + 1, M + 201)):
        tail += psi(x + m * h, h)
    return (h / psi_hat(xi0, h)) * (alias + tail)


def table1_gaussian(x, mu: float, a: np.ndarray):
    """Re sum_{j=-L}^{L} a_j / (ix + mu + ij), a indexed j = -L..L."""
    L = (len(a) - 1) // 2
    z = 1j * np.asarray(x, dtype=np.float64)
    out = np.zeros(z.shape, dtype=np.complex128)
    for j in range(-L, L + 1):
        out += a[j + L] / (z + mu + 1j * j)
    return out.real
