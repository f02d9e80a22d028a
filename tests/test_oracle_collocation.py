"""Pins of the oracle's discretisation, solves and time step.

P4   Chebyshev differentiation is exact on polynomials of degree <= p-1.
P5'  manufactured variable-coefficient solution: the assembled collocation
     system reproduces a smooth exact solution to spectral accuracy, and the
     error falls as p grows (pins the operator, its scaling, the flux rows).
P8   resolvent identity: the scalar elliptic reduction equals a dense solve
     of the first-order system (tau L_h - alpha) (u, v) = (u0, v0).
P9   closed-form Dirichlet eigenmodes for constant c: the step reproduces
     cos / sin propagation to n * delta + discretisation error.
P11  brute force on tiny grids: the step equals V R(tau Lambda) V^{-1} u.
P12  conjugate folding equals the full 2M+1 pole sum.
"""
import numpy as np
import pytest

from oracle import cheb, dense
from oracle import collocation as col
from workloads import fields, layout
from workloads.rational import calibrated_fit


@pytest.mark.parametrize("p", [4, 6, 10, 12, 16])
def test_cheb_diff_exact_on_polynomials(p):
    x = cheb.nodes(p)
    D = cheb.diff_matrix(p)
    for m in range(p):
        exact = m * x ** (m - 1) if m else 0 * x
        assert np.abs(D @ x ** m - exact).max() < 1e-13 * p ** 2


@pytest.mark.parametrize("p", [4, 7, 12, 16])
def test_layout_nodes_match_oracle_nodes(p):
    np.testing.assert_allclose(layout.lobatto_unit(p), cheb.unit_nodes(p),
                               rtol=0, atol=1e-15)


def test_layout_shared_nodes_are_bitwise_equal():
    mesh = layout.Mesh(3, 2, 6, 0.0, 1.5, -1.0, 0.0)
    X, Y = layout.element_nodes(mesh)
    p = mesh.p
    Xa, Xb = X[0].reshape(p, p), X[1].reshape(p, p)     # neighbours in x
    assert np.array_equal(Xa[:, -1], Xb[:, 0])
    Ya, Yb = Y[0].reshape(p, p), Y[3].reshape(p, p)     # neighbours in y
    assert np.array_equal(Ya[-1, :], Yb[0, :])


def _manufactured(X, Y):
    """u = sin(pi x) sin(pi y) e^{x/2}, c^2 = 1 + 0.3 x^2 + 0.2 sin(3 y)
    on [0,1]^2; returns u, c^2 and div(c^2 grad u)."""
    s, c = np.sin, np.cos
    pi = np.pi
    E = np.exp(X / 2)
    u = s(pi * X) * s(pi * Y) * E
    ux = (pi * c(pi * X) + 0.5 * s(pi * X)) * s(pi * Y) * E
    uy = pi * s(pi * X) * c(pi * Y) * E
    uxx = (-pi * pi * s(pi * X) + pi * c(pi * X) + 0.25 * s(pi * X)) * s(pi * Y) * E
    uyy = -pi * pi * u
    k = 1 + 0.3 * X ** 2 + 0.2 * s(3 * Y)
    kx, ky = 0.6 * X, 0.6 * c(3 * Y)
    return u, k, k * (uxx + uyy) + kx * ux + ky * uy


@pytest.mark.parametrize("nex,ney", [(4, 4), (2, 4), (4, 1), (1, 1)])
def test_manufactured_solution_spectral_accuracy(nex, ney):
    sigma = (4.3 + 3.0j) ** 2 / 0.25
    errs = []
    for p in (5, 7, 9, 16):
        mesh = layout.Mesh(nex, ney, p)
        X, Y = layout.element_nodes(mesh)
        u, c2, Ku = _manufactured(X, Y)
        grid = col.make_grid(nex, ney, p)
        K, P = col.assemble(grid, c2)
        m = layout.interior_mask(p)
        g = (Ku - sigma * u)[:, m].reshape(-1)
        y = col.ShiftedSolver(K, P, sigma, grid.n_int).solve_interior(g)
        errs.append(np.abs(y - u[:, m].reshape(-1)).max())
    assert errs[2] < errs[1] < errs[0]
    assert errs[3] < 1e-8, errs


def test_manufactured_solution_on_a_stretched_domain():
    """hx != hy and a domain other than the unit square."""
    sigma = 50.0 + 20.0j
    p = 14
    mesh = layout.Mesh(2, 4, p, 0.0, 2.0, 0.0, 1.0)
    X, Y = layout.element_nodes(mesh)
    s = np.sin
    u = s(np.pi * X / 2) * s(np.pi * Y)            # zero on the boundary
    c2 = 1.0 + 0.0 * X
    Ku = -(np.pi ** 2) * (0.25 + 1.0) * u
    grid = col.make_grid(2, 4, p, 0.0, 2.0, 0.0, 1.0)
    K, P = col.assemble(grid, c2)
    m = layout.interior_mask(p)
    y = col.ShiftedSolver(K, P, sigma, grid.n_int).solve_interior(
        (Ku - sigma * u)[:, m].reshape(-1))
    assert np.abs(y - u[:, m].reshape(-1)).max() < 1e-10


@pytest.fixture(scope="module")
def const_c_stepper():
    mesh = layout.Mesh(4, 4, 12)
    fit = calibrated_fit(41)
    st = col.WaveStepper(col.make_grid(4, 4, 12), np.ones((16, 144)), 0.5,
                         fit.alpha, fit.b, folded=True)
    return mesh, fit, st


@pytest.mark.parametrize("k,l", [(1, 1), (1, 2), (2, 2), (3, 1), (2, 3)])
def test_dirichlet_eigenmodes_closed_form(const_c_stepper, k, l):
    mesh, fit, st = const_c_stepper
    X, Y = layout.interior_nodes(mesh)
    om = np.pi * np.hypot(k, l)
    assert st.tau * om <= fit.X
    phi = fields.dirichlet_mode(X, Y, k, l)
    n = 6
    # displacement data: u = cos(w t) phi, v = -w sin(w t) phi
    u, v = st.run(phi, 0 * phi, n)
    t = n * st.tau
    tol = n * 1e-10 + 5e-10
    assert np.abs(u - np.cos(om * t) * phi).max() < tol
    assert np.abs(v / om + np.sin(om * t) * phi).max() < tol
    # velocity data: u = sin(w t)/w phi, v = cos(w t) phi
    u, v = st.run(0 * phi, phi, n)
    assert np.abs(u * om - np.sin(om * t) * phi).max() < tol
    assert np.abs(v - np.cos(om * t) * phi).max() < tol


def test_out_of_band_mode_is_not_amplified(const_c_stepper):
    """A mode with |tau w| >> X is outside the fitted band; eq. RM_prop2
    keeps it bounded over many steps."""
    mesh, fit, st = const_c_stepper
    X, Y = layout.interior_nodes(mesh)
    phi = fields.dirichlet_mode(X, Y, 9, 8)
    u, v = st.run(phi, 0 * phi, 20)
    assert np.abs(u).max() <= 1.0 + 1e-6


@pytest.fixture(scope="module")
def tiny():
    """2 x 2 elements, p = 6, variable c: L_h is 128 x 128."""
    mesh = layout.Mesh(2, 2, 6)
    X, Y = layout.element_nodes(mesh)
    c2 = fields.smooth_speed(X, Y) ** 2
    grid = col.make_grid(2, 2, 6)
    fit = calibrated_fit(21)
    st = col.WaveStepper(grid, c2, 0.5, fit.alpha, fit.b, folded=False)
    L = dense.first_order_operator(dense.interior_operator(st.K, grid.n_int))
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal(grid.n_int)
    v0 = rng.standard_normal(grid.n_int)
    return st, L, fit, u0, v0


def test_resolvent_identity_dense(tiny):
    st, L, fit, u0, v0 = tiny
    for m in (-3, 0, 2, st.M):
        a = fit.alpha[m + st.M]
        u, v = st.resolvent(m, u0, v0)
        ud, vd = dense.dense_resolvent(L, st.tau, a, u0, v0)
        scale = max(np.abs(ud).max(), np.abs(vd).max())
        assert np.abs(u - ud).max() < 1e-12 * scale
        assert np.abs(v - vd).max() < 1e-12 * scale


def test_interior_operator_spectrum_is_negative_real(tiny):
    st, L, fit, u0, v0 = tiny
    n = L.shape[0] // 2
    kap = np.linalg.eigvals(L[n:, :n])
    assert np.abs(kap.imag).max() < 1e-6 * np.abs(kap).max()
    assert kap.real.max() < 0


def test_step_equals_eigendecomposition(tiny):
    st, L, fit, u0, v0 = tiny
    u, v = st.run(u0, v0, 3)
    ue, ve = dense.eig_step(L, st.tau, fit.alpha, fit.b, u0, v0, n_steps=3)
    scale = max(np.abs(ue).max(), np.abs(ve).max())
    assert np.abs(ue.imag).max() < 1e-10 * scale
    assert np.abs(u - ue.real).max() < 1e-10 * scale
    assert np.abs(v - ve.real).max() < 1e-10 * scale


def test_step_tracks_exact_propagator_in_band(tiny):
    """For data made of in-band eigenvectors, R(tau L) ~ e^{tau L} to delta."""
    st, L, fit, u0, v0 = tiny
    lam, V = np.linalg.eig(L)
    keep = np.abs(st.tau * lam.imag) <= fit.X
    assert keep.sum() >= 2
    w = np.zeros(lam.size, dtype=complex)
    w[keep] = 1.0
    y = (V @ w).real
    n = L.shape[0] // 2
    u, v = st.step(y[:n], y[n:])
    ue, ve = dense.eig_exact(L, st.tau, y[:n], y[n:])
    assert np.abs(u - ue.real).max() < 1e-8 * np.abs(y).max()


def test_folding_equals_full_pole_sum():
    mesh = layout.Mesh(4, 2, 8)
    X, Y = layout.element_nodes(mesh)
    c2 = fields.smooth_speed(X, Y) ** 2
    grid = col.make_grid(4, 2, 8)
    fit = calibrated_fit(21)
    full = col.WaveStepper(grid, c2, 0.5, fit.alpha, fit.b, folded=False)
    fold = col.WaveStepper(grid, c2, 0.5, fit.alpha, fit.b, folded=True)
    Xi, Yi = layout.interior_nodes(mesh)
    u0 = fields.gaussian_pulse(Xi, Yi, 3)
    v0 = 0.5 * fields.gaussian_pulse(Xi, Yi, 4)
    a = full.step(u0, v0)
    b = fold.step(u0, v0)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-14 * np.abs(x).max()
    # over several steps the rounding-level differences are carried between
    # u and v by factors up to tau * omega_max, so compare more loosely
    a = full.run(u0, v0, 3)
    b = fold.run(u0, v0, 3)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-11 * np.abs(x).max()
