"""Mesh, node coordinates and state layout (the data contract of the C-ABI).

The domain [x0,x1]x[y0,y1] is split into nex x ney equal rectangles
("elements"); element e = ex + nex*ey.  Each element carries a p x p
tensor grid of Chebyshev-Lobatto nodes (paper section 2.2), ordered in
ascending coordinate, x index fastest: node (i, j) has local index i + p*j.

The time-stepper state lives on element-interior nodes only
(1 <= i, j <= p-2); with q = p-2, interior node (i, j) of element e has
index  e*q*q + (i-1) + q*(j-1)  inside one field.  A state buffer holds
[rhs][field][element][q*q] doubles.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Mesh:
    nex: int
    ney: int
    p: int
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0

    @property
    def q(self) -> int:
        return self.p - 2

    @property
    def n_el(self) -> int:
        return self.nex * self.ney

    @property
    def n_int(self) -> int:
        """Interior nodes per field (the state length of one field)."""
        return self.n_el * self.q * self.q

    @property
    def hx(self) -> float:
        return (self.x1 - self.x0) / self.nex

    @property
    def hy(self) -> float:
        return (self.y1 - self.y0) / self.ney


def lobatto_unit(p: int) -> np.ndarray:
    """Chebyshev-Lobatto points mapped to [0, 1], ascending; ends exact."""
    k = np.arange(p, dtype=np.float64)
    return np.sin(0.5 * np.pi * k / (p - 1)) ** 2


def element_nodes(mesh: Mesh) -> tuple[np.ndarray, np.ndarray]:
    """Coordinates of all p*p nodes of every element.

    Returns X, Y with shape (n_el, p*p) in the local order i + p*j.
    Nodes shared by neighbouring elements get bit-identical coordinates.
    """
    t = lobatto_unit(mesh.p)
    ex = np.arange(mesh.nex, dtype=np.float64)
    ey = np.arange(mesh.ney, dtype=np.float64)
    xs = mesh.x0 + mesh.hx * (ex[:, None] + t[None, :])      # (nex, p)
    ys = mesh.y0 + mesh.hy * (ey[:, None] + t[None, :])      # (ney, p)
    X = np.empty((mesh.n_el, mesh.p * mesh.p))
    Y = np.empty_like(X)
    for jy in range(mesh.ney):
        for ix in range(mesh.nex):
            e = ix + mesh.nex * jy
            X[e] = np.tile(xs[ix], mesh.p)
            Y[e] = np.repeat(ys[jy], mesh.p)
    return X, Y


def interior_mask(p: int) -> np.ndarray:
    """Boolean mask over the p*p local nodes selecting the interior ones."""
    m = np.zeros((p, p), dtype=bool)          # indexed [j, i]
    m[1:-1, 1:-1] = True
    return m.reshape(-1)


def interior_nodes(mesh: Mesh) -> tuple[np.ndarray, np.ndarray]:
    """Coordinates of the state entries of one field, flattened (n_int,)."""
    X, Y = element_nodes(mesh)
    m = interior_mask(mesh.p)
    return X[:, m].reshape(-1), Y[:, m].reshape(-1)
