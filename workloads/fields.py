"""Wave-speed fields and initial states, all seeded and synthetic.

The paper's experiments use smooth analytic coefficients and initial data
(section 4); the workloads here follow the same spirit with the shapes of
the benchmark configurations:

* a smooth analytic speed 1 + 0.25 sin(2 pi x) sin(2 pi y);
* Gaussian random fields with a squared-exponential covariance of
  correlation length ell, drawn as random Fourier features (Rahimi and
  Recht, 2007) from numpy's PCG64 with a fixed seed;
* Gaussian pulses exp(-|x - x0|^2 / (2 s^2)) centred at a seeded point;
* Dirichlet eigenmodes sin(k pi x) sin(l pi y).

Every function returns values sampled at given coordinates; nothing here
knows about the discretisation beyond those coordinates.
"""
from __future__ import annotations

import numpy as np


def smooth_speed(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """c(x, y) = 1 + 0.25 sin(2 pi x) sin(2 pi y)."""
    return 1.0 + 0.25 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)


class FourierFeatureField:
    """Zero-mean, unit-variance random field with covariance
    exp(-|x - x'|^2 / (2 ell^2)), approximated by n_features random
    Fourier features: g(x) = sqrt(2/K) sum_k cos(w_k . x + phi_k),
    w_k ~ N(0, ell^-2 I), phi_k ~ U[0, 2 pi)."""

    def __init__(self, seed: int, ell: float = 0.1, n_features: int = 1024):
        rng = np.random.default_rng(seed)
        self.w = rng.normal(0.0, 1.0 / ell, size=(n_features, 2))
        self.phi = rng.uniform(0.0, 2 * np.pi, size=n_features)
        self.scale = np.sqrt(2.0 / n_features)

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        flat_x, flat_y = x.reshape(-1), y.reshape(-1)
        ux, ix = np.unique(flat_x, return_inverse=True)
        uy, iy = np.unique(flat_y, return_inverse=True)
        if ux.size * uy.size <= 4 * flat_x.size:
            # points on a tensor grid: cos(a + b) = cos a cos b - sin a sin b
            # with a = w1 x + phi, b = w2 y makes the sum one matrix product
            a = np.outer(ux, self.w[:, 0]) + self.phi
            b = np.outer(uy, self.w[:, 1])
            grid = np.cos(a) @ np.cos(b).T - np.sin(a) @ np.sin(b).T
            return (self.scale * grid[ix, iy]).reshape(x.shape)
        out = np.empty(flat_x.shape)
        step = 65536
        for s in range(0, flat_x.size, step):
            arg = (np.outer(flat_x[s:s + step], self.w[:, 0])
                   + np.outer(flat_y[s:s + step], self.w[:, 1]) + self.phi)
            out[s:s + step] = self.scale * np.cos(arg).sum(axis=1)
        return out.reshape(x.shape)


def clipped_lognormal_speed(x, y, seed: int, mean=np.log(2.0), std=0.35,
                            lo=1.0, hi=3.0, ell=0.1) -> np.ndarray:
    """c = clip(exp(mean + std * g), lo, hi), g a unit Gaussian field."""
    g = FourierFeatureField(seed, ell)(x, y)
    return np.clip(np.exp(mean + std * g), lo, hi)


def contrast_lognormal_speed(x, y, seed: int, contrast=4.0, ell=0.1):
    """c = exp(g'), g' = the field g affinely rescaled over the given points
    to [0, ln contrast], so min c = 1 and max c = contrast exactly."""
    g = FourierFeatureField(seed, ell)(x, y)
    g = (g - g.min()) / (g.max() - g.min())
    return np.exp(g * np.log(contrast))


def pulse_centre(seed: int) -> tuple[float, float]:
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.25, 0.75, size=2)
    return float(c[0]), float(c[1])


def gaussian_pulse(x, y, seed: int, width=0.05) -> np.ndarray:
    """exp(-|x - x0|^2 / (2 width^2)) with x0 ~ U[0.25, 0.75]^2 (seeded)."""
    cx, cy = pulse_centre(seed)
    return np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * width ** 2))


def dirichlet_mode(x, y, k: int, l: int) -> np.ndarray:
    return np.sin(k * np.pi * x) * np.sin(l * np.pi * y)


def wall_modes_state(x, y, seed: int, kmax: float = 30.0):
    """Random-phase smooth shallow-water state on [0,1]^2 built from the
    slip-wall basis (n . v = 0 on every side of the unit square):
        eta0 = sum a_k  cos(k1 pi x) cos(k2 pi y),
        v1   = sum a'_k sin(k1 pi x) cos(k2 pi y),
        v2   = sum a''_k cos(k1 pi x) sin(k2 pi y),
    over integer k = (k1, k2) >= 0 with 0 < |k| <= kmax, |a| = |k|^-2 (shell
    energy ~ k^-3) and independent random signs from the seed.  All three
    fields are divided by max |eta0| over the given points.
    Returns (v1, v2, eta0), each shaped like x."""
    rng = np.random.default_rng(seed)
    kk = np.arange(int(np.floor(kmax)) + 1, dtype=np.float64)
    K1, K2 = np.meshgrid(kk, kk, indexing="ij")
    kmod = np.hypot(K1, K2)
    keep = (kmod > 0) & (kmod <= kmax)
    amp = np.where(keep, 1.0 / np.where(keep, kmod, 1.0) ** 2, 0.0)
    a0, a1, a2 = (amp * rng.choice([-1.0, 1.0], size=amp.shape) for _ in range(3))
    xs, ys = np.asarray(x, dtype=np.float64).reshape(-1), np.asarray(y, dtype=np.float64).reshape(-1)
    cx, sx_ = np.cos(np.pi * kk[:, None] * xs[None, :]), np.sin(np.pi * kk[:, None] * xs[None, :])
    cy, sy_ = np.cos(np.pi * kk[:, None] * ys[None, :]), np.sin(np.pi * kk[:, None] * ys[None, :])
    eta = np.einsum("an,an->n", cx, a0 @ cy)
    v1 = np.einsum("an,an->n", sx_, a1 @ cy)
    v2 = np.einsum("an,an->n", cx, a2 @ sy_)
    scale = 1.0 / np.abs(eta).max()
    shape = np.shape(x)
    return ((v1 * scale).reshape(shape), (v2 * scale).reshape(shape),
            (eta * scale).reshape(shape))
