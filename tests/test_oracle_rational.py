"""Pins of the oracle's rational-function code against the paper.

P1  Table 1 (section 3.2): the printed mu and a_j approximate the Gaussian
    psi_1 to about 7e-13 in the form Re sum a_j / (ix + mu + ij).
P2  Gaussian sums (section 3.1 and the appendix bound).
P3  the residue sets fed to the stepper satisfy eq. RM_prop1 (error <= delta
    on |x| <= X) and eq. RM_prop2 (|R| <= 1 on the real line, to 1e-6),
    with exact conjugate symmetry of the poles and residues.
"""
import os

import numpy as np
import pytest

from conftest import GOLDEN
from oracle import rational as orat
from workloads import rational as wrat


def load_table1():
    mu, a = None, {}
    with open(os.path.join(GOLDEN, "table1_gaussian_rational.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            if tok[0] == "mu":
                mu = float(tok[1])
            else:
                a[int(tok[0])] = complex(float(tok[1]), float(tok[2]))
    L = max(a)
    return mu, np.array([a[j] for j in range(-L, L + 1)])


def test_table1_reproduces_printed_error():
    mu, a = load_table1()
    assert a.size == 23
    x = np.linspace(-60.0, 60.0, 240001)
    err = np.abs(orat.table1_gaussian(x, mu, a) - orat.psi(x)).max()
    # "about 7e-13" over the real line, and below 1e-12 (section 3.2)
    assert 5e-13 < err < 1e-12, err
    # beyond the fitted window the error keeps decaying (|R| -> 0)
    xf = np.geomspace(60.0, 1e6, 2000)
    assert np.abs(orat.table1_gaussian(xf, mu, a)).max() < 1e-12


def test_table1_rejects_the_other_printed_form():
    """The intro's 2 Re sum a_j / (ix - (mu + ij)) form is not the one the
    coefficients were made for: it misses psi_1 by O(1) (reading of the
    garbled display in section 3)."""
    mu, a = load_table1()
    x = np.linspace(-30.0, 30.0, 6001)
    L = 11
    other = np.zeros(x.shape, dtype=complex)
    for j in range(-L, L + 1):
        other += a[j + L] / (1j * x - (mu + 1j * j))
    err = np.abs(2 * other.real - orat.psi(x)).max()
    assert err > 1e-2


def test_gaussian_sum_within_appendix_bound():
    M, h = 50, 1.0
    x = np.linspace(-60.0, 60.0, 4801)
    approx = orat.gaussian_sum_exp(x, M, h)
    err = np.abs(approx - np.exp(1j * x))
    bound = orat.gaussian_sum_bound(x, M, h)
    rounding = 1e-14 * np.e * (2 * M + 1)
    assert np.all(err <= bound + rounding)
    inner = np.abs(x) <= M - 12
    assert err[inner].max() < 1e-11
    # near the ends of the window the truncation term dominates and is large
    assert err[np.abs(x) >= 59.0].max() > 1e-3


def test_gaussian_psi_hat_is_the_fourier_transform():
    """psi_h^ (xi) = int psi_h(x) exp(-2 pi i x xi) dx, by quadrature."""
    h = 0.7
    x = np.linspace(-40, 40, 160001)
    dx = x[1] - x[0]
    for xi in (0.0, 0.1, 0.3):
        num = (orat.psi(x, h) * np.exp(-2j * np.pi * x * xi)).sum() * dx
        assert abs(num - orat.psi_hat(xi, h)) < 1e-10


@pytest.mark.parametrize("npoles", sorted(wrat.CALIBRATED))
def test_calibrated_fit_meets_rm_properties(npoles):
    fit = wrat.calibrated_fit(npoles)
    M = fit.M
    assert fit.alpha.size == npoles
    np.testing.assert_array_equal(fit.alpha[::-1], np.conj(fit.alpha))
    np.testing.assert_array_equal(fit.b[::-1], np.conj(fit.b))
    assert fit.b[M].imag == 0.0
    assert orat.fit_error(fit.alpha, fit.b, fit.X) <= 1e-10
    assert orat.max_modulus(fit.alpha, fit.b) <= 1.0 + 1e-6


def test_rational_eval_symmetry_and_decay():
    fit = wrat.calibrated_fit(21)
    x = np.linspace(-50, 50, 1001)
    r = orat.R_eval(fit.alpha, fit.b, 1j * x)
    np.testing.assert_allclose(r[::-1], np.conj(r), rtol=0, atol=1e-13)
    # proper rational function: x R(ix) -> sum_m b_m / i
    big = 1e9
    lim = orat.R_eval(fit.alpha, fit.b, np.array([1j * big]))[0] * 1j * big
    assert abs(lim - fit.b.sum()) < 1e-6 * np.abs(fit.b).sum()
