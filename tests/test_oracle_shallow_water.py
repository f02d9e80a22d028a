"""Pins of the shallow-water oracle (slip walls).

* f = 0: Neumann modes eta = cos(k pi x) cos(l pi y), v = 0 evolve as
  eta(t) = cos(w t) eta0, v(t) = (c sin(w t)/w) grad(eta0), w = c pi |(k, l)|.
* f != 0: the geostrophic state eta = sin(k pi x) sin(l pi y),
  v = (c/f)(-d_y eta, d_x eta) is steady and satisfies the wall condition.
* the conjugate-folded pole sum equals the full one.
* the interior-line differentiation and end-point interpolation are exact on
  polynomials of degree < q.
"""
import numpy as np
import pytest

from oracle import cheb
from oracle import shallow_water as sw
from workloads import layout
from workloads.rational import calibrated_fit


def test_interior_line_operators_exact_on_polynomials():
    for p in (6, 10, 12):
        xq = cheb.nodes(p)[1:-1]
        Dq = sw.interp_diff_matrices(xq)
        lo, hi = sw.end_weights(xq, -1.0), sw.end_weights(xq, 1.0)
        for m in range(p - 2):
            f = xq ** m
            assert np.abs(Dq @ f - (m * xq ** (m - 1) if m else 0 * xq)).max() < 1e-11
            assert abs(lo @ f - (-1.0) ** m) < 1e-11
            assert abs(hi @ f - 1.0) < 1e-11


def _mode_error(p, k, l, n=5, tau=0.3):
    g = sw.SWGrid(4, 4, p)
    fit = calibrated_fit(41)
    st = sw.SWStepper(g, 0.0, 1.0, tau, fit.alpha, fit.b)
    X, Y = layout.interior_nodes(layout.Mesh(4, 4, p))
    eta0 = np.cos(k * np.pi * X) * np.cos(l * np.pi * Y)
    om = np.pi * np.hypot(k, l)
    assert tau * om <= fit.X
    z = 0 * eta0
    v1, v2, eta = st.run(z, z, eta0, n)
    t = n * tau
    gx = -k * np.pi * np.sin(k * np.pi * X) * np.cos(l * np.pi * Y)
    gy = -l * np.pi * np.cos(k * np.pi * X) * np.sin(l * np.pi * Y)
    amp = np.sin(om * t) / om
    return max(np.abs(eta - np.cos(om * t) * eta0).max(),
               np.abs(v1 - amp * gx).max() / max(1, k),
               np.abs(v2 - amp * gy).max() / max(1, l))


@pytest.mark.parametrize("k,l", [(1, 0), (1, 1), (2, 1), (0, 3)])
def test_neumann_modes_f0(k, l):
    """Closed form to discretisation accuracy: the error falls spectrally
    with p (the velocity derivatives use q = p-2 point lines)."""
    errs = [_mode_error(p, k, l) for p in (6, 8, 12)]
    assert errs[2] < errs[1] < errs[0] or errs[1] < 1e-9
    assert errs[2] < 1e-7, errs


def _geo_error(p, f, k, l):
    g = sw.SWGrid(4, 2, p)
    fit = calibrated_fit(41)
    st = sw.SWStepper(g, f, 1.0, 0.3, fit.alpha, fit.b)
    X, Y = layout.interior_nodes(layout.Mesh(4, 2, p))
    eta = np.sin(k * np.pi * X) * np.sin(l * np.pi * Y)
    ex = k * np.pi * np.cos(k * np.pi * X) * np.sin(l * np.pi * Y)
    ey = l * np.pi * np.sin(k * np.pi * X) * np.cos(l * np.pi * Y)
    v1, v2 = -ey / f, ex / f
    a1, a2, a3 = st.run(v1, v2, eta, 4)
    scale = max(np.abs(v1).max(), 1.0)
    return max(np.abs(a3 - eta).max(), np.abs(a1 - v1).max() / scale,
               np.abs(a2 - v2).max() / scale)


@pytest.mark.parametrize("f,k,l,p_fine,bound", [(1.0, 1, 1, 12, 1e-8), (2.5, 1, 2, 14, 5e-8)])
def test_geostrophic_state_is_steady(f, k, l, p_fine, bound):
    """Steady to discretisation accuracy, falling spectrally with p."""
    errs = [_geo_error(p, f, k, l) for p in (8, 10, p_fine)]
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < bound, errs


def test_folded_equals_full_pole_sum():
    g = sw.SWGrid(2, 2, 8)
    fit = calibrated_fit(21)
    rng = np.random.default_rng(5)
    X, Y = layout.interior_nodes(layout.Mesh(2, 2, 8))
    v1 = np.sin(np.pi * X) * np.cos(2 * np.pi * Y) * 0.3
    v2 = np.cos(np.pi * X) * np.sin(np.pi * Y) * 0.2
    eta = np.cos(np.pi * X) * np.cos(np.pi * Y) + 0.1 * rng.standard_normal(X.size)
    a = sw.SWStepper(g, 1.0, 1.0, 0.5, fit.alpha, fit.b, folded=False).step(v1, v2, eta)
    b = sw.SWStepper(g, 1.0, 1.0, 0.5, fit.alpha, fit.b, folded=True).step(v1, v2, eta)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-13 * np.abs(x).max() * np.abs(fit.b).sum()
