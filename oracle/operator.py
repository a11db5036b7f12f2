"""Finite-difference Poisson matrix on the masked lattice (oracle).

Paper, Section 2.  At an unknown x every axis i contributes the 1-D difference
(-u(x - h e_i) + 2 u(x) - u(x + h e_i)) / h_i^2 (eq. 7pt-star).  When a neighbour lies
outside the domain, its value is replaced by an extrapolation through the wall point
at fraction s (homogeneous wall data, g = 0):

* constant (eq. const_extrapol):  u(x') = 0;
* linear   (eq. lin_extrapol):    u(x') = (1 - 1/s) u(x);
* quadratic, other neighbour x'' inside (eq. quad_extrapol):
      u(x') = 2(s - 1)/s u(x) - (s - 1)/(s + 1) u(x'');
* quadratic, both neighbours outside with fractions s and t (eq. quad_extrapol1):
      u(x') = (s - 1)(t + 1)/(s t) u(x),   u(x'') = (s + 1)(t - 1)/(s t) u(x).

Each axis is handled on its own and the contributions add up (the paper applies the
rules in every direction in which the point is near the wall).  The substitution is
carried out literally below, term by term, so that a reader can match it against the
equations; the resulting per-axis rows are what the tests pin against closed forms.

Open ends (Section 2, eq. inlet): on a domain with Robin ends, a node x on an end plane
has its outside z-neighbour x' replaced by u(x') = u(x'') - (2 h_z / d) u(x), with x''
the inside z-neighbour and d half the length of the pipe.  Reading: the rows of the end
planes are divided by 2 (and so is their right-hand side).  This leaves the solution
unchanged and keeps the constant and linear rules symmetric, as Section 2 states they
are.

Scaling (end of Section 2): with D = diag(A) the system A x = b is replaced by
(D^-1/2 A D^-1/2) y = D^-1/2 b, x = D^-1/2 y.
"""
from __future__ import annotations

import dataclasses
from typing import Tuple

import numpy as np
import scipy.sparse as sp

from .grid import Domain

CONST, LIN, QUAD = 0, 1, 2


@dataclasses.dataclass
class System:
    """Assembled system over the unknowns of a domain, in box-lexicographic order."""

    dom: Domain
    variant: int
    A: sp.csr_matrix          # unscaled matrix (end-plane rows of open ends halved)
    idx: np.ndarray           # box-linear index of each unknown
    sigma: np.ndarray         # D^-1/2
    As: sp.csr_matrix         # scaled matrix D^-1/2 A D^-1/2
    rho: np.ndarray = None    # row factor applied to A and b (1/2 on open-end rows)

    @property
    def n(self) -> int:
        return self.idx.size

    def gather(self, box: np.ndarray) -> np.ndarray:
        return np.asarray(box, dtype=np.float64).reshape(-1)[self.idx]

    def scatter(self, v: np.ndarray) -> np.ndarray:
        out = np.zeros(self.dom.nx * self.dom.ny * self.dom.nz)
        out[self.idx] = v
        return out.reshape(self.dom.nz, self.dom.ny, self.dom.nx)


def _axis_terms(variant: int, in_m: np.ndarray, in_p: np.ndarray, s_m: np.ndarray,
                s_p: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Coefficients (times h^2) of u(x), u(x - h e) and u(x + h e) for one axis.

    Start from -u(x-) + 2 u(x) - u(x+) and substitute every outside neighbour by its
    extrapolation; the returned neighbour coefficients are zero for outside neighbours.
    """
    c_self = np.full(in_m.shape, 2.0)
    c_m = np.where(in_m, -1.0, 0.0)
    c_p = np.where(in_p, -1.0, 0.0)
    out_m, out_p = ~in_m, ~in_p
    if variant == CONST:
        # u(x') = g = 0: the outside term simply disappears.
        return c_self, c_m, c_p
    if variant == LIN:
        # -u(x') = -(1 - 1/s) u(x), for each outside side independently.
        c_self = c_self - np.where(out_m, 1.0 - 1.0 / s_m, 0.0)
        c_self = c_self - np.where(out_p, 1.0 - 1.0 / s_p, 0.0)
        return c_self, c_m, c_p
    if variant != QUAD:
        raise ValueError(variant)
    one_m = out_m & in_p
    one_p = out_p & in_m
    both = out_m & out_p
    # One side outside: -u(x') = -2(s-1)/s u(x) + (s-1)/(s+1) u(x'').
    c_self = c_self - np.where(one_m, 2.0 * (s_m - 1.0) / s_m, 0.0)
    c_p = c_p + np.where(one_m, (s_m - 1.0) / (s_m + 1.0), 0.0)
    c_self = c_self - np.where(one_p, 2.0 * (s_p - 1.0) / s_p, 0.0)
    c_m = c_m + np.where(one_p, (s_p - 1.0) / (s_p + 1.0), 0.0)
    # Both outside (s on the minus side, t on the plus side).
    s, t = s_m, s_p
    c_self = c_self - np.where(both, (s - 1.0) * (t + 1.0) / (s * t), 0.0)
    c_self = c_self - np.where(both, (s + 1.0) * (t - 1.0) / (s * t), 0.0)
    return c_self, c_m, c_p


def _robin_sides(dom: Domain, ks: np.ndarray):
    """Open-end sides of each unknown: its -z / +z neighbour is the ghost plane."""
    if dom.robin_d <= 0.0:
        z = np.zeros(ks.shape, dtype=bool)
        return z, z
    return ks - 1 == 0, ks + 1 == dom.nz - 1


def _robin_z_terms(h: float, d: float, out_m: np.ndarray, out_p: np.ndarray, c_self, c_m, c_p):
    """z-coefficients (times h^2) of end-plane rows, eq. inlet substituted into
    -u(x') + 2 u(x) - u(x''):  (2 + 2h/d) u(x) - 2 u(x'')."""
    if not np.any(out_m | out_p):
        return c_self, c_m, c_p
    if np.any(out_m & out_p):
        raise ValueError("an open end needs an unknown z-neighbour on the other side")
    c_self = np.where(out_m | out_p, 2.0 + 2.0 * h / d, c_self)
    c_p = np.where(out_m, -2.0, c_p)
    c_m = np.where(out_p, -2.0, c_m)
    return c_self, c_m, c_p


def assemble(dom: Domain, variant: int) -> System:
    """Unscaled and scaled matrices of the discrete Poisson problem."""
    nx, ny, nz = dom.nx, dom.ny, dom.nz
    mask = dom.mask
    ks, js, is_ = np.nonzero(mask)
    idx = (is_ + nx * (js + ny * ks)).astype(np.int64)
    n = idx.size
    compact = np.full(nx * ny * nz, -1, dtype=np.int64)
    compact[idx] = np.arange(n)
    rob_m, rob_p = _robin_sides(dom, ks)
    rho = np.where(rob_m | rob_p, 0.5, 1.0)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], []
    diag = np.zeros(n)
    for axis in range(3):
        d_m, d_p = 2 * axis, 2 * axis + 1
        step = [0, 0, 0]
        step[axis] = 1
        dz, dy, dx = step[2], step[1], step[0]
        in_m = mask[ks - dz, js - dy, is_ - dx]
        in_p = mask[ks + dz, js + dy, is_ + dx]
        s_m = dom.frac[d_m, ks, js, is_]
        s_p = dom.frac[d_p, ks, js, is_]
        c_self, c_m, c_p = _axis_terms(variant, in_m, in_p, s_m, s_p)
        if axis == 2:
            c_self, c_m, c_p = _robin_z_terms(dom.h[2], dom.robin_d, rob_m, rob_p,
                                              c_self, c_m, c_p)
        inv_h2 = 1.0 / (dom.h[axis] * dom.h[axis])
        diag += rho * c_self * inv_h2
        lin_step = dx + nx * (dy + ny * dz)
        for c, sgn, inside in ((c_m, -1, in_m), (c_p, 1, in_p)):
            sel = np.nonzero(inside)[0]
            rows.append(sel)
            cols.append(compact[idx[sel] + sgn * lin_step])
            vals.append(rho[sel] * c[sel] * inv_h2)
    vals.insert(0, diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    A.sum_duplicates()
    A.eliminate_zeros()
    D = A.diagonal()
    sigma = 1.0 / np.sqrt(D)
    S = sp.diags(sigma)
    As = (S @ A @ S).tocsr()
    As.sort_indices()
    return System(dom, variant, A, idx, sigma, As, rho)


def diagonal(dom: Domain, variant: int):
    """Diagonal of A at every unknown (box-lexicographic order) without assembling A.

    Same per-axis rule as ``assemble``; used to scale right-hand sides of grids too large
    to assemble in a test.  Returns (box indices of the unknowns, diagonal).
    """
    nx, ny = dom.nx, dom.ny
    ks, js, is_ = np.nonzero(dom.mask)
    diag = np.zeros(ks.size)
    rob_m, rob_p = _robin_sides(dom, ks)
    rho = np.where(rob_m | rob_p, 0.5, 1.0)
    for axis in range(3):
        step = [0, 0, 0]
        step[axis] = 1
        dx, dy, dz = step
        in_m = dom.mask[ks - dz, js - dy, is_ - dx]
        in_p = dom.mask[ks + dz, js + dy, is_ + dx]
        s_m = dom.frac[2 * axis, ks, js, is_]
        s_p = dom.frac[2 * axis + 1, ks, js, is_]
        c_self, c_m, c_p = _axis_terms(variant, in_m, in_p, s_m, s_p)
        if axis == 2:
            c_self, _, _ = _robin_z_terms(dom.h[2], dom.robin_d, rob_m, rob_p, c_self, c_m, c_p)
        diag += rho * c_self / (dom.h[axis] * dom.h[axis])
    return (is_ + nx * (js + ny * ks)).astype(np.int64), diag


def scaled_residual(dom: Domain, variant: int, x_box: np.ndarray, b_box: np.ndarray):
    """D^-1/2 rho (b - A x) at every unknown (box-lexicographic order), without assembling A.

    The rows are those of ``assemble`` (the same per-axis rule, open-end rows and their
    right-hand side multiplied by rho = 1/2); each axis adds its centre and neighbour
    terms over all unknowns at once.  For grids too large to assemble (tens of millions
    of unknowns): the scaled true residual of a solution, whose norm over ||D^-1/2 rho b||
    is the relative residual of Section 5's stopping rule.  Returns (residual, ||b~||).
    """
    nx, ny = dom.nx, dom.ny
    ks, js, is_ = np.nonzero(dom.mask)
    xf = np.asarray(x_box, dtype=np.float64).reshape(-1)
    bf = np.asarray(b_box, dtype=np.float64).reshape(-1)
    lin = (is_ + nx * (js + ny * ks)).astype(np.int64)
    rob_m, rob_p = _robin_sides(dom, ks)
    rho = np.where(rob_m | rob_p, 0.5, 1.0)
    diag = np.zeros(ks.size)
    ax = np.zeros(ks.size)
    x0 = xf[lin]
    for axis in range(3):
        step = [0, 0, 0]
        step[axis] = 1
        dx, dy, dz = step
        in_m = dom.mask[ks - dz, js - dy, is_ - dx]
        in_p = dom.mask[ks + dz, js + dy, is_ + dx]
        s_m = dom.frac[2 * axis, ks, js, is_]
        s_p = dom.frac[2 * axis + 1, ks, js, is_]
        c_self, c_m, c_p = _axis_terms(variant, in_m, in_p, s_m, s_p)
        if axis == 2:
            c_self, c_m, c_p = _robin_z_terms(dom.h[2], dom.robin_d, rob_m, rob_p,
                                              c_self, c_m, c_p)
        inv_h2 = 1.0 / (dom.h[axis] * dom.h[axis])
        lin_step = dx + nx * (dy + ny * dz)
        x_m = np.where(in_m, xf[lin - lin_step], 0.0)
        x_p = np.where(in_p, xf[lin + lin_step], 0.0)
        diag += rho * c_self * inv_h2
        ax += rho * (c_self * x0 + c_m * x_m + c_p * x_p) * inv_h2
    sig = 1.0 / np.sqrt(diag)
    bs = sig * rho * bf[lin]
    return bs - sig * ax, float(np.linalg.norm(bs))


def scaled_rhs(sys_: System, b_box: np.ndarray) -> np.ndarray:
    """D^-1/2 b over the unknowns (b of the open-end rows halved with the rows)."""
    return sys_.sigma * sys_.rho * sys_.gather(b_box)


def unscale(sys_: System, y: np.ndarray) -> np.ndarray:
    """x = D^-1/2 y over the unknowns."""
    return sys_.sigma * y
