"""Linearised rotating shallow water with slip walls (O1, plain definition).

Equations (paper section 2.1, example 1, with c = sqrt(gH) made explicit):
    v_t = -f J v + c grad(eta),   eta_t = c div(v),   J = [[0, 1], [-1, 0]],
on a rectangle with slip walls n . v = 0.

Resolvent (the section 2.1 reduction, worked for this form): with
a = alpha/tau, s = a^2 + f^2 and primes meaning "divided by tau",
    (tau L - alpha)(v, eta) = (v0, eta0)
  <=> v = A (c grad(eta) - v0'),  A = (a I + f J)^{-1} = (a I - f J)/s,
      (Lap - s/c^2) eta = (s/(c^2 a)) eta0' + div(v0')/c - (f/(c a)) curl(v0'),
with curl(w) = d_x w_2 - d_y w_1, and the wall condition n . v = 0 becomes
the oblique condition
      a d_n eta - f d_t eta = (a n.v0' - f t.v0') / c,   t = (-n_2, n_1).
(The paper's A_alpha is written for periodic boundaries; on walls the
tangential term is what makes the slip condition exact.)

Discretisation readings (the paper is periodic and does not treat walls):
  * the state (v1, v2, eta) lives on element-interior nodes;
  * eta is an unknown at interior, interface and wall nodes (corners are
    referenced by no equation); PDE rows at interior nodes, flux rows
    (d_n eta(a) + d_n eta(b) = 0) at interface nodes, oblique rows at wall
    nodes, where d_n eta is the element's spectral derivative along the full
    p-point line and d_t eta the derivative along the wall side through its
    q = p-2 non-corner nodes;
  * derivatives of v0 inside an element use the q-point differentiation
    along interior lines, and v0 at a wall node is the value at the wall of
    the degree q-1 polynomial through the q interior values on the line
    normal to the wall;
  * grad(eta) at interior nodes uses the element's p-point lines.

Step: (v, eta) <- sum_m b_m (tau L - alpha_m)^{-1} (v, eta) (section 1.2).

Pinned by: Neumann modes cos(k pi x) cos(l pi y) for f = 0 (closed form) and
the geostrophic steady state for f != 0 (tests).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import cheb


def interp_diff_matrices(x: np.ndarray):
    """Differentiation matrix of the polynomial interpolating values at the
    distinct nodes x, evaluated at the same nodes (barycentric form)."""
    n = x.size
    c = np.array([np.prod([x[k] - x[j] for j in range(n) if j != k]) for k in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (c[i] / c[j]) / (x[i] - x[j])
        D[i, i] = -D[i].sum()
    return D


def end_weights(x: np.ndarray, x_end: float) -> np.ndarray:
    """Lagrange basis of the nodes x evaluated at x_end."""
    w = np.ones(x.size)
    for k in range(x.size):
        for j in range(x.size):
            if j != k:
                w[k] *= (x_end - x[j]) / (x[k] - x[j])
    return w


class SWGrid:
    """Unknown numbering: element interiors, then interface nodes (vertical
    then horizontal interfaces), then wall nodes (left, right, bottom, top
    walls, element by element along each wall)."""

    def __init__(self, nex, ney, p, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
        self.nex, self.ney, self.p = nex, ney, p
        self.q = p - 2
        self.hx = (x1 - x0) / nex
        self.hy = (y1 - y0) / ney
        q = self.q
        self.n_int = nex * ney * q * q
        self.n_vert = (nex - 1) * ney * q
        self.n_horz = nex * (ney - 1) * q
        self.base_wall = self.n_int + self.n_vert + self.n_horz
        self.n_wall = 2 * (nex + ney) * q
        self.n_unknowns = self.base_wall + self.n_wall

    def wall_index(self, side: int, k: int, t: int) -> int:
        """side 0 left (x = x0), 1 right, 2 bottom, 3 top; k = element index
        along the wall, t = node along the element side."""
        q, nex, ney = self.q, self.nex, self.ney
        off = [0, ney * q, 2 * ney * q, 2 * ney * q + nex * q][side]
        return self.base_wall + off + k * q + t

    def unknown(self, ex, ey, i, j):
        p, q = self.p, self.q
        last = p - 1
        if 0 < i < last and 0 < j < last:
            return (ex + self.nex * ey) * q * q + (i - 1) + q * (j - 1)
        if (i in (0, last)) and (j in (0, last)):
            raise ValueError("corner nodes are not unknowns")
        if i == 0 or i == last:
            vx = ex - 1 if i == 0 else ex
            if vx < 0:
                return self.wall_index(0, ey, j - 1)
            if vx >= self.nex - 1:
                return self.wall_index(1, ey, j - 1)
            return self.n_int + (vx + (self.nex - 1) * ey) * q + (j - 1)
        hy_ = ey - 1 if j == 0 else ey
        if hy_ < 0:
            return self.wall_index(2, ex, i - 1)
        if hy_ >= self.ney - 1:
            return self.wall_index(3, ex, i - 1)
        return self.n_int + self.n_vert + (ex + self.nex * hy_) * q + (i - 1)


def assemble_sw(g: SWGrid):
    """Return (K, P, O): K holds the Laplacian PDE rows and the flux rows,
    P selects the PDE rows (shift), and for the wall rows the two parts of
    the oblique condition: O_n (element normal derivative) and O_t
    (tangential derivative), so that the wall rows are a O_n - f O_t."""
    p, q = g.p, g.q
    D = cheb.diff_matrix(p)
    xq = cheb.nodes(p)[1:-1]
    Dq = interp_diff_matrices(xq)
    sx, sy = 2.0 / g.hx, 2.0 / g.hy
    n = g.n_unknowns
    rows, cols, vals = [], [], []
    On_r, On_c, On_v = [], [], []
    Ot_r, Ot_c, Ot_v = [], [], []

    def put(L, r, c, v):
        L[0].append(r)
        L[1].append(c)
        L[2].append(v)

    K_ = (rows, cols, vals)
    D2 = D @ D
    for ey in range(g.ney):
        for ex in range(g.nex):
            for j in range(1, p - 1):
                for i in range(1, p - 1):
                    r = g.unknown(ex, ey, i, j)
                    for k in range(p):
                        put(K_, r, g.unknown(ex, ey, k, j), sx * sx * D2[i, k])
                        put(K_, r, g.unknown(ex, ey, i, k), sy * sy * D2[j, k])
    for ey in range(g.ney):
        for vx in range(g.nex - 1):
            for j in range(1, p - 1):
                r = g.unknown(vx, ey, p - 1, j)
                for k in range(p):
                    put(K_, r, g.unknown(vx, ey, k, j), sx * D[p - 1, k])
                    put(K_, r, g.unknown(vx + 1, ey, k, j), -sx * D[0, k])
    for hy_ in range(g.ney - 1):
        for ex in range(g.nex):
            for i in range(1, p - 1):
                r = g.unknown(ex, hy_, i, p - 1)
                for l in range(p):
                    put(K_, r, g.unknown(ex, hy_, i, l), sy * D[p - 1, l])
                    put(K_, r, g.unknown(ex, hy_ + 1, i, l), -sy * D[0, l])
    On, Ot = (On_r, On_c, On_v), (Ot_r, Ot_c, Ot_v)
    # wall rows: outward normal derivative along the element's line, and the
    # tangential derivative t . grad along the wall side's q nodes
    for side in range(4):
        nel = g.ney if side < 2 else g.nex
        for k in range(nel):
            if side == 0:
                ex, ey, lo, xn = 0, k, True, True
            elif side == 1:
                ex, ey, lo, xn = g.nex - 1, k, False, True
            elif side == 2:
                ex, ey, lo, xn = k, 0, True, False
            else:
                ex, ey, lo, xn = k, g.ney - 1, False, False
            sc = sx if xn else sy
            st = sy if xn else sx
            row_d = D[0] if lo else D[p - 1]
            nsign = -1.0 if lo else 1.0
            # t = (-n2, n1): left (0,-1) -> -d_y, right (0,1) -> +d_y,
            # bottom (1,0) -> +d_x, top (-1,0) -> -d_x
            tsign = {0: -1.0, 1: 1.0, 2: 1.0, 3: -1.0}[side]
            for t in range(q):
                r = g.wall_index(side, k, t)
                for l in range(p):
                    node = (l, t + 1) if xn else (t + 1, l)
                    if (node[0] in (0, p - 1)) and (node[1] in (0, p - 1)):
                        continue
                    put(On, r, g.unknown(ex, ey, *node), nsign * sc * row_d[l])
                for u in range(q):
                    put(Ot, r, g.wall_index(side, k, u), tsign * st * Dq[t, u])
    K = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    K.sum_duplicates()
    pd = np.zeros(n)
    pd[:g.n_int] = 1.0
    On_m = sp.csr_matrix((On_v, (On_r, On_c)), shape=(n, n))
    Ot_m = sp.csr_matrix((Ot_v, (Ot_r, Ot_c)), shape=(n, n))
    return K, sp.diags(pd), On_m, Ot_m


class SWStepper:
    """exp(tau L) (v1, v2, eta) ~ sum_m b_m (tau L - alpha_m)^{-1} (v1, v2, eta)."""

    def __init__(self, g: SWGrid, f: float, gH: float, tau: float, alpha, b,
                 folded: bool = True):
        self.g, self.f, self.c, self.tau = g, float(f), float(np.sqrt(gH)), float(tau)
        self.alpha = np.asarray(alpha, dtype=np.complex128)
        self.b = np.asarray(b, dtype=np.complex128)
        self.M = (self.alpha.size - 1) // 2
        self.folded = folded
        self.K, self.P, self.On, self.Ot = assemble_sw(g)
        p, q = g.p, g.q
        self.D = cheb.diff_matrix(p)
        xq = cheb.nodes(p)[1:-1]
        self.Dq = interp_diff_matrices(xq)
        self.w_lo = end_weights(xq, -1.0)
        self.w_hi = end_weights(xq, 1.0)
        wall = np.zeros(g.n_unknowns)
        wall[g.base_wall:] = 1.0
        self.Wsel = sp.diags(wall)
        ms = range(0, self.M + 1) if folded else range(-self.M, self.M + 1)
        self.lu = {}
        for m in ms:
            a = self.alpha[m + self.M] / self.tau
            s = a * a + self.f ** 2
            B = (self.K - (s / self.c ** 2) * self.P + a * self.On - self.f * self.Ot)
            self.lu[m] = spla.splu(B.astype(np.complex128).tocsc())

    # -- element-local helpers (interior fields shaped (n_el, q, q) as [e][j][i]) --
    def _grid(self, x):
        g = self.g
        return x.reshape(g.ney, g.nex, g.q, g.q)

    def interior_derivs(self, w):
        """d/dx and d/dy of an interior field by q-point differentiation along
        interior lines (physical scaling)."""
        g = self.g
        W = w.reshape(g.nex * g.ney, g.q, g.q)              # [e][j][i]
        dx = np.einsum('ik,ejk->eji', self.Dq, W) * (2.0 / g.hx)
        dy = np.einsum('jk,eki->eji', self.Dq, W) * (2.0 / g.hy)
        return dx.reshape(-1), dy.reshape(-1)

    def wall_values(self, v1, v2):
        """n . v and t . v at every wall node (wall-unknown order)."""
        g = self.g
        q = g.q
        V1 = v1.reshape(g.ney, g.nex, q, q)
        V2 = v2.reshape(g.ney, g.nex, q, q)
        nv = np.zeros(g.n_wall)
        tv = np.zeros(g.n_wall)
        for side in range(4):
            nel = g.ney if side < 2 else g.nex
            for k in range(nel):
                for t in range(q):
                    if side == 0:      # x = x0, line along x at row t
                        e1 = V1[k, 0, t, :] @ self.w_lo
                        e2 = V2[k, 0, t, :] @ self.w_lo
                        n_, t_ = -e1, -e2
                    elif side == 1:
                        e1 = V1[k, g.nex - 1, t, :] @ self.w_hi
                        e2 = V2[k, g.nex - 1, t, :] @ self.w_hi
                        n_, t_ = e1, e2
                    elif side == 2:    # y = y0, line along y at column t
                        e1 = V1[0, k, :, t] @ self.w_lo
                        e2 = V2[0, k, :, t] @ self.w_lo
                        n_, t_ = -e2, e1
                    else:
                        e1 = V1[g.ney - 1, k, :, t] @ self.w_hi
                        e2 = V2[g.ney - 1, k, :, t] @ self.w_hi
                        n_, t_ = e2, -e1
                    idx = g.wall_index(side, k, t) - g.base_wall
                    nv[idx], tv[idx] = n_, t_
        return nv, tv

    def grad_eta(self, eta_full):
        """grad(eta) at interior nodes from all unknowns (p-point lines)."""
        g = self.g
        p, q = g.p, g.q
        gx = np.zeros(g.n_int, dtype=complex)
        gy = np.zeros(g.n_int, dtype=complex)
        for ey in range(g.ney):
            for ex in range(g.nex):
                for j in range(1, p - 1):
                    for i in range(1, p - 1):
                        r = g.unknown(ex, ey, i, j)
                        gx[r] = sum(self.D[i, k] * eta_full[g.unknown(ex, ey, k, j)]
                                    for k in range(p)) * (2.0 / g.hx)
                        gy[r] = sum(self.D[j, k] * eta_full[g.unknown(ex, ey, i, k)]
                                    for k in range(p)) * (2.0 / g.hy)
        return gx, gy

    def resolvent(self, m, v1, v2, eta):
        g, f, c, tau = self.g, self.f, self.c, self.tau
        a = self.alpha[m + self.M] / tau
        s = a * a + f * f
        d1x, d1y = self.interior_derivs(v1)
        d2x, d2y = self.interior_derivs(v2)
        div = (d1x + d2y) / tau
        curl = (d2x - d1y) / tau
        rhs = np.zeros(g.n_unknowns, dtype=complex)
        rhs[:g.n_int] = (s / (c * c * a)) * eta / tau + div / c - (f / (c * a)) * curl
        nv, tv = self.wall_values(v1, v2)
        rhs[g.base_wall:] = (a * nv - f * tv) / (tau * c)
        full = self.lu[m].solve(rhs)
        gx, gy = self.grad_eta(full)
        w1 = c * gx - v1 / tau
        w2 = c * gy - v2 / tau
        # A w = (a w - f J w)/s, J w = (w2, -w1)
        return (a * w1 - f * w2) / s, (a * w2 + f * w1) / s, full[:g.n_int]

    def step(self, v1, v2, eta):
        M = self.M
        out = [np.zeros(v1.shape, dtype=complex) for _ in range(3)]
        ms = range(0, M + 1) if self.folded else range(-M, M + 1)
        for m in ms:
            res = self.resolvent(m, v1, v2, eta)
            w = self.b[m + M]
            for k in range(3):
                if self.folded and m > 0:
                    out[k] += 2.0 * (w * res[k]).real
                else:
                    out[k] += w * res[k]
        return tuple(o.real.copy() for o in out)

    def run(self, v1, v2, eta, n):
        for _ in range(n):
            v1, v2, eta = self.step(v1, v2, eta)
        return v1, v2, eta
