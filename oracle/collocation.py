"""Global multidomain collocation system and the rational time step (O1).

Discretisation (paper section 2.2).  The domain is tiled by nex x ney
rectangles, each with a p x p Chebyshev tensor grid.  Unknowns are the
values at
  * element-interior nodes, where the PDE is collocated with spectral
    differentiation on the element's own grid, and
  * interface nodes (non-corner nodes of an edge shared by two elements),
    where the outward normal derivatives of the two neighbours must cancel.
Nodes on the outer boundary carry the homogeneous Dirichlet value 0 and
are not unknowns.  Corner nodes of elements are referenced by no equation
(the operator has no mixed derivative) and are not unknowns either.

Operator.  For u_t = v, v_t = div(c^2 grad u) (wave equation, first-order
form), the elliptic operator is K = div(c^2 grad .), collocated in the
nested form Dx C^2 Dx + Dy C^2 Dy with C^2 = diag(c^2 at the nodes).
Because c^2 is one value per shared node, flux continuity c^2 du/dn
(either side) reduces to du/dn(a) + du/dn(b) = 0.

Resolvent (section 2.1, worked here for this first-order form; the paper
does the same substitution for its (w, z, v) form in eqs. w-and-z /
v-for-inhomog):
    (tau L - alpha) (u, v) = (u0, v0)
  <=> (K - sigma) u = g,  sigma = (alpha/tau)^2,  g = (alpha u0 + tau v0)/tau^2,
      v = (alpha u + u0) / tau.

Time step (section 1.2, eq. def_RM and the sum before it):
    (u, v) <- sum_{m=-M}^{M} b_m (tau L - alpha_m)^{-1} (u, v),
the pole sum is formed over all 2M+1 poles (the definition); ``folded``
uses the conjugate symmetry of section 3.3 (only m >= 0 solved).

Every solve is a sparse LU (SuperLU) of the whole assembled system: the
plain definition that the hierarchical solver reproduces up to rounding.

Pinned by: closed-form Dirichlet eigenmodes (constant c), a manufactured
variable-c solution, the tiny-grid eigendecomposition of ``dense``, and
the resolvent identity (tests).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import cheb


@dataclasses.dataclass
class Grid:
    nex: int
    ney: int
    p: int
    hx: float
    hy: float

    @property
    def q(self):
        return self.p - 2

    @property
    def n_el(self):
        return self.nex * self.ney

    @property
    def n_int(self):
        return self.n_el * self.q * self.q

    @property
    def n_vert(self):             # interface nodes on vertical interfaces
        return (self.nex - 1) * self.ney * self.q

    @property
    def n_horz(self):
        return self.nex * (self.ney - 1) * self.q

    @property
    def n_unknowns(self):
        return self.n_int + self.n_vert + self.n_horz

    def unknown(self, ex: int, ey: int, i: int, j: int) -> int:
        """Global unknown of local node (i, j) of element (ex, ey);
        -1 for an outer-boundary node.  Corners are never asked for."""
        p, q = self.p, self.q
        last = p - 1
        if 0 < i < last and 0 < j < last:
            return (ex + self.nex * ey) * q * q + (i - 1) + q * (j - 1)
        if (i in (0, last)) and (j in (0, last)):
            raise ValueError("corner nodes are not unknowns")
        if i == 0 or i == last:                 # vertical edge, position j
            vx = ex - 1 if i == 0 else ex       # interface between vx, vx+1
            if vx < 0 or vx >= self.nex - 1:
                return -1
            return self.n_int + (vx + (self.nex - 1) * ey) * q + (j - 1)
        hy_ = ey - 1 if j == 0 else ey          # horizontal edge, position i
        if hy_ < 0 or hy_ >= self.ney - 1:
            return -1
        return self.n_int + self.n_vert + (ex + self.nex * hy_) * q + (i - 1)


def make_grid(nex, ney, p, x0=0.0, x1=1.0, y0=0.0, y1=1.0) -> Grid:
    return Grid(nex, ney, p, (x1 - x0) / nex, (y1 - y0) / ney)


def assemble(grid: Grid, c2: np.ndarray):
    """Return (K, P): the sparse operator with PDE rows div(c^2 grad) and
    flux rows, and the diagonal selector P of the PDE rows, so that the
    shifted system is B(sigma) = K - sigma P.

    c2: (n_el, p*p) values of c^2 at every node, local order i + p*j.
    """
    p, q = grid.p, grid.q
    D = cheb.diff_matrix(p)
    sx, sy = 2.0 / grid.hx, 2.0 / grid.hy
    rows, cols, vals = [], [], []

    def put(r, c, v):
        if c >= 0:
            rows.append(r)
            cols.append(c)
            vals.append(v)

    for ey in range(grid.ney):
        for ex in range(grid.nex):
            e = ex + grid.nex * ey
            cc = c2[e].reshape(p, p)            # [j, i]
            for j in range(1, p - 1):
                Mx = sx * sx * (D @ (cc[j, :][:, None] * D))     # along x
                for i in range(1, p - 1):
                    r = grid.unknown(ex, ey, i, j)
                    for k in range(p):
                        put(r, grid.unknown(ex, ey, k, j), Mx[i, k])
            for i in range(1, p - 1):
                My = sy * sy * (D @ (cc[:, i][:, None] * D))     # along y
                for j in range(1, p - 1):
                    r = grid.unknown(ex, ey, i, j)
                    for l in range(p):
                        put(r, grid.unknown(ex, ey, i, l), My[j, l])
    # flux rows: outward normal derivatives of the two neighbours cancel
    for ey in range(grid.ney):
        for vx in range(grid.nex - 1):          # a = (vx, ey) left, b right
            for j in range(1, p - 1):
                r = grid.unknown(vx, ey, p - 1, j)
                for k in range(p):
                    put(r, grid.unknown(vx, ey, k, j), sx * D[p - 1, k])
                    put(r, grid.unknown(vx + 1, ey, k, j), -sx * D[0, k])
    for hy_ in range(grid.ney - 1):
        for ex in range(grid.nex):              # a = (ex, hy_) below, b above
            for i in range(1, p - 1):
                r = grid.unknown(ex, hy_, i, p - 1)
                for l in range(p):
                    put(r, grid.unknown(ex, hy_, i, l), sy * D[p - 1, l])
                    put(r, grid.unknown(ex, hy_ + 1, i, l), -sy * D[0, l])
    n = grid.n_unknowns
    K = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    K.sum_duplicates()
    pdiag = np.zeros(n)
    pdiag[:grid.n_int] = 1.0
    return K, sp.diags(pdiag)


class ShiftedSolver:
    """Sparse LU of B(sigma) = K - sigma P for one shift sigma."""

    def __init__(self, K, P, sigma: complex, n_int: int):
        B = (K - sigma * P).astype(np.complex128).tocsc()
        self.lu = spla.splu(B)
        self.n = K.shape[0]
        self.n_int = n_int

    def solve_interior(self, g: np.ndarray) -> np.ndarray:
        """Solve B u = [g; 0]; return u at the interior nodes."""
        rhs = np.zeros(self.n, dtype=np.complex128)
        rhs[:self.n_int] = g
        return self.lu.solve(rhs)[:self.n_int]

    def solve_full(self, f: np.ndarray) -> np.ndarray:
        return self.lu.solve(np.asarray(f, dtype=np.complex128))


class WaveStepper:
    """exp(tau L) (u, v) ~ sum_m b_m (tau L - alpha_m)^{-1} (u, v) for the
    wave equation u_t = v, v_t = div(c^2 grad u), homogeneous Dirichlet."""

    def __init__(self, grid: Grid, c2: np.ndarray, tau: float,
                 alpha: np.ndarray, b: np.ndarray, folded: bool = False):
        self.grid, self.tau = grid, float(tau)
        self.alpha = np.asarray(alpha, dtype=np.complex128)
        self.b = np.asarray(b, dtype=np.complex128)
        self.M = (self.alpha.size - 1) // 2
        self.folded = folded
        self.K, self.P = assemble(grid, c2)
        ms = range(0, self.M + 1) if folded else range(-self.M, self.M + 1)
        self.solvers = {m: ShiftedSolver(self.K, self.P,
                                         (self.alpha[m + self.M] / tau) ** 2,
                                         grid.n_int) for m in ms}

    def resolvent(self, m: int, u0, v0):
        """(tau L - alpha_m)^{-1} (u0, v0) on the interior nodes."""
        a, tau = self.alpha[m + self.M], self.tau
        u = self.solvers[m].solve_interior((a * u0 + tau * v0) / tau ** 2)
        return u, (a * u + u0) / tau

    def step(self, u0: np.ndarray, v0: np.ndarray):
        M = self.M
        u1 = np.zeros(u0.shape, dtype=np.complex128)
        v1 = np.zeros(u0.shape, dtype=np.complex128)
        if not self.folded:
            for m in range(-M, M + 1):
                um, vm = self.resolvent(m, u0, v0)
                u1 += self.b[m + M] * um
                v1 += self.b[m + M] * vm
            return u1.real.copy(), v1.real.copy()
        # conjugate folding: for real data the m and -m terms are conjugate
        um, vm = self.resolvent(0, u0, v0)
        u1 += self.b[M] * um
        v1 += self.b[M] * vm
        for m in range(1, M + 1):
            um, vm = self.resolvent(m, u0, v0)
            u1 += 2.0 * (self.b[m + M] * um).real
            v1 += 2.0 * (self.b[m + M] * vm).real
        return u1.real.copy(), v1.real.copy()

    def run(self, u0, v0, n_steps: int):
        u, v = np.array(u0, dtype=np.float64), np.array(v0, dtype=np.float64)
        for _ in range(n_steps):
            u, v = self.step(u, v)
        return u, v
