"""Lattice, unknowns and wall distances of a beam-pipe domain (oracle).

Paper, Section 2: the lattice is the set of points whose coordinates are integer
multiples of the spacing; a lattice point is an unknown when it lies inside the
domain.  For a point x next to the curved wall, the wall point between x and its
outside neighbour x' = x - h e_i is x* = x - s h e_i with 0 < s <= 1 (Figure
"boundary"); s = 1 means x' itself lies on the wall.

Readings where the paper leaves a choice open:
* the lattice spans the bounding box of the pipe with n nodes per axis, both ends
  included, so h = extent / (n - 1); node i of an axis of half-extent a sits at
  a * (2 i - (n - 1)) / (n - 1);
* "inside" is strict (points on the wall are not unknowns), the two end caps are
  Dirichlet walls, so planes k = 0 and k = nz - 1 never hold unknowns, and neither
  do the faces of the box;
* a wall fraction within 1e-12 of 1 is taken as exactly 1.

This file is the oracle's own geometry; the GPU library computes its domain with
separate code, and the tests compare the two.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Tuple

import numpy as np

CYLINDER, ELLIPSE, BOXBORE = 0, 1, 2
S_SNAP = 1e-12
ON_WALL = 1e-12  # a point inside only by this relative margin lies on the wall

# Direction order used for wall fractions: -x, +x, -y, +y, -z, +z.
DIRS = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


@dataclasses.dataclass
class Domain:
    """Discrete domain on an (nz, ny, nx) box.

    mask[k, j, i]      True where the node is an unknown.
    frac[d][k, j, i]   wall fraction s in direction d for unknowns whose neighbour in
                       that direction is not an unknown; 1.0 everywhere else.
    """

    nx: int
    ny: int
    nz: int
    h: Tuple[float, float, float]
    mask: np.ndarray
    frac: np.ndarray  # (6, nz, ny, nx)
    robin_d: float = 0.0  # > 0: open ends (Robin), the box carries one ghost plane per end

    @property
    def n_unknowns(self) -> int:
        return int(self.mask.sum())


def coords(half: float, n: int) -> np.ndarray:
    m = 2.0 * np.arange(n, dtype=np.float64) - (n - 1)
    return half * m / (n - 1)


def _inside_xy(kind: int, a: float, b: float, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    if kind == CYLINDER:
        return X * X + Y * Y < a * a * (1.0 - ON_WALL)
    if kind == ELLIPSE:
        return (X / a) ** 2 + (Y / b) ** 2 < 1.0 - ON_WALL
    raise ValueError(kind)


def _in_bore(X: np.ndarray, Y: np.ndarray, r: float) -> np.ndarray:
    return X * X + Y * Y < r * r * (1.0 - ON_WALL)


def build(kind: int, a: float, b: float, length: float, nx: int, ny: int, nz: int,
          bore_r: float = 0.0, cavity_half_len: float = 0.0, robin: bool = False) -> Domain:
    """Classify every box node and compute wall fractions (vectorised where simple).

    With ``robin`` the two end planes z = -L/2 and z = +L/2 of the lattice are open
    boundary (Section 2, the Robin condition on Gamma_2): their nodes inside the
    cross-section are unknowns, and the box gains one empty ghost plane beyond each end, so
    the returned domain has nz + 2 planes with the lattice's plane k at box plane k + 1.
    """
    if robin:
        inner = build(kind, a, b, length, nx, ny, nz, bore_r, cavity_half_len)
        z = coords(0.5 * length, nz)
        Y, X = np.meshgrid(coords(b, ny), coords(a, nx), indexing="ij")
        ends = np.zeros((ny, nx), dtype=bool)
        ends[1:-1, 1:-1] = True
        if kind in (CYLINDER, ELLIPSE):
            ends &= _inside_xy(kind, a, b, X, Y)
        else:  # the bore, and the cavity if it reaches the ends
            keep = 1.0 - ON_WALL
            cav = (np.abs(X) < a * keep) & (np.abs(Y) < b * keep) & (0.5 * length < cavity_half_len * keep)
            ends &= cav | _in_bore(X, Y, bore_r)
        mask = np.zeros((nz + 2, ny, nx), dtype=bool)
        mask[1:-1] = inner.mask
        mask[1] = mask[-2] = ends
        frac = np.ones((6, nz + 2, ny, nx))
        frac[:, 1:-1] = inner.frac
        # wall fractions of the end-plane nodes in x and y (z: the open boundary)
        for kb, zv in ((1, z[0]), (nz, z[-1])):
            js, is_ = np.nonzero(ends)
            for d in range(4):
                dy, dx = DIRS[d][1], DIRS[d][0]
                sel = np.nonzero(~ends[js + dy, is_ + dx])[0]
                if sel.size:
                    j, i = js[sel], is_[sel]
                    frac[d, kb, j, i] = _wall_fraction(
                        kind, a, b, length, bore_r, cavity_half_len, coords(a, nx)[i],
                        coords(b, ny)[j], np.full(sel.size, zv), inner.h, d)
            frac[4:, kb] = 1.0
        # the planes next to the ends now have unknown neighbours there (no wall)
        frac[4, 2][mask[1]] = 1.0
        frac[5, nz - 1][mask[nz]] = 1.0
        return Domain(nx, ny, nz + 2, inner.h, mask, frac, 0.5 * length)
    x = coords(a, nx)
    y = coords(b, ny)
    z = coords(0.5 * length, nz)
    h = (2.0 * a / (nx - 1), 2.0 * b / (ny - 1), length / (nz - 1))
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    interior_idx = np.zeros((nz, ny, nx), dtype=bool)
    interior_idx[1:-1, 1:-1, 1:-1] = True
    if kind in (CYLINDER, ELLIPSE):
        mask = _inside_xy(kind, a, b, X, Y) & interior_idx
    elif kind == BOXBORE:
        keep = 1.0 - ON_WALL
        cav = (np.abs(X) < a * keep) & (np.abs(Y) < b * keep) & (np.abs(Z) < cavity_half_len * keep)
        bore = _in_bore(X, Y, bore_r)
        mask = (cav | bore) & interior_idx
    else:
        raise ValueError(kind)

    frac = np.ones((6, nz, ny, nx), dtype=np.float64)
    ks, js, is_ = np.nonzero(mask)
    for d, (dx, dy, dz) in enumerate(DIRS):
        nb = mask[ks + dz, js + dy, is_ + dx]
        sel = np.nonzero(~nb)[0]
        if sel.size == 0:
            continue
        k, j, i = ks[sel], js[sel], is_[sel]
        frac[d, k, j, i] = _wall_fraction(kind, a, b, length, bore_r, cavity_half_len,
                                          x[i], y[j], z[k], h, d)
    return Domain(nx, ny, nz, h, mask, frac)


def _wall_fraction(kind, a, b, length, bore_r, cav_half, xs, ys, zs, h, d) -> np.ndarray:
    """Distance, in units of h, from unknowns at (xs, ys, zs) to the wall in direction d."""
    axis = d // 2
    sign = -1.0 if d % 2 == 0 else 1.0
    pos = (xs, ys, zs)[axis]
    # End of the open interval that the domain occupies on each grid line.
    if kind in (CYLINDER, ELLIPSE):
        if axis == 2:
            end = np.full(pos.shape, 0.5 * length)
        elif kind == CYLINDER:
            other = ys if axis == 0 else xs
            end = np.sqrt(np.maximum(a * a - other * other, 0.0))
        elif axis == 0:
            end = a * np.sqrt(np.maximum(1.0 - (ys / b) ** 2, 0.0))
        else:
            end = b * np.sqrt(np.maximum(1.0 - (xs / a) ** 2, 0.0))
    else:  # BOXBORE
        in_cavity_z = np.abs(zs) < cav_half * (1.0 - ON_WALL)
        if axis == 2:
            in_bore = _in_bore(xs, ys, bore_r)
            end = np.where(in_bore, 0.5 * length, cav_half)
        else:
            other = ys if axis == 0 else xs
            chord = np.sqrt(np.maximum(bore_r * bore_r - other * other, 0.0))
            end = np.where(in_cavity_z, a if axis == 0 else b, chord)
    wall = sign * end
    s = np.abs(wall - pos) / h[axis]
    s = np.where(s > 1.0 - S_SNAP, 1.0, s)
    if not np.all(s > 0.0):
        raise ValueError(f"non-positive wall fraction in direction {d}")
    return s


def from_shape(shape, nx: int, ny: int, nz: int, robin: bool = False) -> Domain:
    """Build from a ``workloads.Shape``-like object (kind, a, b, length, ...)."""
    return build(shape.kind, shape.a, shape.b, shape.length, nx, ny, nz,
                 getattr(shape, "bore_r", 0.0), getattr(shape, "cavity_half_len", 0.0), robin)


def cross_section_count(kind: int, a: float, b: float, nx: int, ny: int) -> int:
    """Number of lattice points strictly inside the cross-section (one z-plane)."""
    X, Y = np.meshgrid(coords(a, nx), coords(b, ny), indexing="xy")
    return int(_inside_xy(kind, a, b, X, Y).sum())


def wall_entries(dom: Domain) -> Dict[str, np.ndarray]:
    """Sparse list (node, dir, s) of wall fractions below 1, box-linear node index."""
    d, k, j, i = np.nonzero(dom.frac < 1.0)
    node = i + dom.nx * (j + dom.ny * k)
    order = np.lexsort((d, node))
    return {"node": node[order].astype(np.int64), "dir": d[order].astype(np.uint8),
            "s": dom.frac[d, k, j, i][order]}
