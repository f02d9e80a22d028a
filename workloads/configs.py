"""The wave-equation workloads as plain, seeded recipes.

Each recipe fixes the mesh, the speed field, the pole count, the step tau,
the initial states and the number of steps.  ``make`` turns a recipe into
arrays (c^2 at every node, the residues, initial states on interior nodes).

Time step for the pulse workloads (a reading; the recipes only say "tau
spanning many wavelengths"): a Gaussian pulse of width s has its spectrum
below k_delta = sqrt(2 ln(1/delta)) / s to relative accuracy delta; with
the largest speed c_max its frequencies stay below Lambda = c_max k_delta,
and tau = X / Lambda puts that band inside the interval |x| <= X on which
the rational function matches e^{ix} (eq. RM_prop1).  tau does not change
the cost of a step, only the shifts of the elliptic solves.
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np

from . import fields, layout
from .rational import RationalFit, calibrated_fit

DELTA = 1e-10


@dataclasses.dataclass(frozen=True)
class WaveRecipe:
    name: str
    mesh: layout.Mesh
    speed: str                  # "smooth" | "clipped_lognormal" | "contrast4" | "const"
    speed_seed: int
    npoles: int
    tau: float | None           # None: tau = X / Lambda (pulse band)
    pulse_seeds: tuple
    pulse_width: float
    n_steps: int

    @property
    def nrhs(self) -> int:
        return len(self.pulse_seeds)


RECIPES = {
    # 4 x 4 elements x 12^2 nodes, c = 1 + 0.25 sin sin, 21 poles, tau = 0.5
    "wave_4x4_p12": WaveRecipe("wave_4x4_p12", layout.Mesh(4, 4, 12), "smooth",
                               0, 21, 0.5, (0,), 0.05, 10),
    # 32 x 32 elements x 16^2 nodes, c = clip(exp(GRF), 1, 3), 101 poles
    "wave_32x32_p16": WaveRecipe("wave_32x32_p16", layout.Mesh(32, 32, 16),
                                 "clipped_lognormal", 1, 101, None, (2,), 0.05, 100),
    # 64 x 64 elements x 10^2 nodes, lognormal contrast 4, 131 poles, 32 RHS
    "wave_64x64_p10": WaveRecipe("wave_64x64_p10", layout.Mesh(64, 64, 10),
                                 "contrast4", 5, 131, None, tuple(range(32)), 0.05, 1000),
}


def speed_function(kind: str, seed: int) -> Callable:
    if kind == "smooth":
        return fields.smooth_speed
    if kind == "const":
        return lambda x, y: np.ones_like(x)
    if kind == "clipped_lognormal":
        return lambda x, y: fields.clipped_lognormal_speed(x, y, seed)
    if kind == "contrast4":
        return lambda x, y: fields.contrast_lognormal_speed(x, y, seed, 4.0)
    raise ValueError(kind)


def pulse_tau(fit: RationalFit, c_max: float, width: float, delta=DELTA) -> float:
    k_delta = np.sqrt(2.0 * np.log(1.0 / delta)) / width
    return fit.X / (c_max * k_delta)


@dataclasses.dataclass
class WaveInputs:
    recipe: WaveRecipe
    mesh: layout.Mesh
    c2: np.ndarray              # (n_el, p*p)
    fit: RationalFit
    tau: float
    u0: np.ndarray              # (nrhs, n_int)
    v0: np.ndarray              # (nrhs, n_int)

    def state(self) -> np.ndarray:
        """[rhs][field][n_int] layout of the C-ABI."""
        return np.ascontiguousarray(np.stack([self.u0, self.v0], axis=1))


def make(recipe: WaveRecipe | str, n_rhs: int | None = None) -> WaveInputs:
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    mesh = recipe.mesh
    X, Y = layout.element_nodes(mesh)
    c = speed_function(recipe.speed, recipe.speed_seed)(X, Y)
    c2 = np.ascontiguousarray(c * c)
    fit = calibrated_fit(recipe.npoles)
    tau = recipe.tau if recipe.tau is not None else pulse_tau(
        fit, float(c.max()), recipe.pulse_width)
    Xi, Yi = layout.interior_nodes(mesh)
    seeds = recipe.pulse_seeds[:n_rhs] if n_rhs else recipe.pulse_seeds
    u0 = np.stack([fields.gaussian_pulse(Xi, Yi, s, recipe.pulse_width) for s in seeds])
    return WaveInputs(recipe, mesh, c2, fit, float(tau), u0, np.zeros_like(u0))


def scaled(recipe: WaveRecipe | str, nex: int, ney: int, p: int | None = None,
           npoles: int | None = None, n_steps: int | None = None) -> WaveRecipe:
    """Same recipe on another mesh (the same field, sampled on new nodes)."""
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    m = recipe.mesh
    return dataclasses.replace(
        recipe, name=f"{recipe.name}@{nex}x{ney}",
        mesh=layout.Mesh(nex, ney, p or m.p, m.x0, m.x1, m.y0, m.y1),
        npoles=npoles or recipe.npoles, n_steps=n_steps or recipe.n_steps)


# ---- shallow water with slip walls ------------------------------------------------


@dataclasses.dataclass(frozen=True)
class SWRecipe:
    """Linearised rotating shallow water on the unit square with slip walls.

    Time step (a reading, as for the pulses): the states hold wavenumbers
    |k| <= kmax (units of pi), whose gravity-inertia frequencies stay below
    omega_max = sqrt(f^2 + gH (kmax pi)^2); tau = X / omega_max keeps them
    inside the interval on which the rational function matches e^{ix}."""
    name: str
    mesh: layout.Mesh
    f: float
    gH: float
    npoles: int
    kmax: float
    seeds: tuple
    n_steps: int

    @property
    def nrhs(self) -> int:
        return len(self.seeds)


SW_RECIPES = {
    # 32 x 32 elements x 12^2 nodes, f = 1, gH = 1, 101 poles, 64 states
    "sw_32x32_p12": SWRecipe("sw_32x32_p12", layout.Mesh(32, 32, 12), 1.0, 1.0, 101, 30.0,
                             tuple(range(64)), 100),
}


@dataclasses.dataclass
class SWInputs:
    recipe: SWRecipe
    mesh: layout.Mesh
    fit: RationalFit
    tau: float
    v1: np.ndarray              # (nrhs, n_int)
    v2: np.ndarray
    eta: np.ndarray

    def state(self) -> np.ndarray:
        """[rhs][field][n_int] layout of the C-ABI, fields (v1, v2, eta)."""
        return np.ascontiguousarray(np.stack([self.v1, self.v2, self.eta], axis=1))


def sw_tau(fit: RationalFit, f: float, gH: float, kmax: float) -> float:
    return fit.X / float(np.sqrt(f * f + gH * (kmax * np.pi) ** 2))


def make_sw(recipe: SWRecipe | str, n_rhs: int | None = None) -> SWInputs:
    if isinstance(recipe, str):
        recipe = SW_RECIPES[recipe]
    mesh = recipe.mesh
    fit = calibrated_fit(recipe.npoles)
    tau = sw_tau(fit, recipe.f, recipe.gH, recipe.kmax)
    Xi, Yi = layout.interior_nodes(mesh)
    seeds = recipe.seeds[:n_rhs] if n_rhs else recipe.seeds
    fs = [fields.wall_modes_state(Xi, Yi, s, recipe.kmax) for s in seeds]
    v1, v2, eta = (np.stack([f[k] for f in fs]) for k in range(3))
    return SWInputs(recipe, mesh, fit, float(tau), v1, v2, eta)


def scaled_sw(recipe: SWRecipe | str, nex: int, ney: int, p: int | None = None,
              npoles: int | None = None, kmax: float | None = None,
              n_steps: int | None = None) -> SWRecipe:
    if isinstance(recipe, str):
        recipe = SW_RECIPES[recipe]
    m = recipe.mesh
    return dataclasses.replace(
        recipe, name=f"{recipe.name}@{nex}x{ney}",
        mesh=layout.Mesh(nex, ney, p or m.p, m.x0, m.x1, m.y0, m.y1),
        npoles=npoles or recipe.npoles, kmax=kmax or recipe.kmax,
        n_steps=n_steps or recipe.n_steps)


# ---- batching form: many wave instances of uneven size ------------------------------


@dataclasses.dataclass(frozen=True)
class BatchRecipe:
    """Wave instances of uneven size stepped together (the batching form).

    Instance i: sides[i % 3] x sides[i % 3] elements of p x p nodes; a
    clipped-lognormal speed with seed i; pole count drawn uniformly from
    `poles` and 1..max_rhs right-hand sides, both from the generator
    seeded 1000 + i; Gaussian pulses with seeds 16 i + j; tau by the pulse
    rule for its own pole count and speed.  Reading: the pole counts are the
    calibrated odd counts in 41..101 (41, 61, 81, 101)."""
    name: str
    n_instances: int
    sides: tuple = (8, 16, 32)
    p: int = 12
    poles: tuple = (41, 61, 81, 101)
    max_rhs: int = 16
    pulse_width: float = 0.05
    n_steps: int = 10


BATCH_RECIPES = {
    "batch_512": BatchRecipe("batch_512", 512),
}


def batch_instance(recipe: BatchRecipe, i: int) -> WaveInputs:
    rng = np.random.default_rng(1000 + i)
    npoles = int(rng.choice(recipe.poles))
    nrhs = int(rng.integers(1, recipe.max_rhs + 1))
    side = recipe.sides[i % len(recipe.sides)]
    rec = WaveRecipe(f"{recipe.name}[{i}]", layout.Mesh(side, side, recipe.p),
                     "clipped_lognormal", i, npoles, None,
                     tuple(16 * i + j for j in range(nrhs)), recipe.pulse_width, recipe.n_steps)
    return make(rec)


def make_batch(recipe: BatchRecipe | str, n: int | None = None) -> list:
    if isinstance(recipe, str):
        recipe = BATCH_RECIPES[recipe]
    return [batch_instance(recipe, i) for i in range(n or recipe.n_instances)]
