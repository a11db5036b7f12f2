"""Particle coupling on either side of the solve: cloud-in-cell deposition and field gather
(oracle).

Paper, Section 1 and Section 4: the particle charges are interpolated to the grid to form
the right-hand side rho, and the field E = -grad(phi) of the solution is interpolated back
to the particles; both use cloud-in-cell (trilinear) weights.

Readings:

* the grid is described by the box dims, the offset of the lattice's plane 0 within the
  box along z (1 with open ends, else 0), the coordinates of lattice node (0, 0, 0) and the
  spacings;
* a particle belongs to the lattice cell [i, i+1) x [j, j+1) x [k, k+1) that contains it
  and gives charge q (1 - f) or q f per axis to the cell's corner nodes (f = the fractional
  position in the cell); the density is the nodal charge divided by h_x h_y h_z; particles
  outside every lattice cell are dropped;
* E at a node is the central difference -(phi(n + e) - phi(n - e)) / (2 h); phi is 0 at
  nodes that are not unknowns (the wall value) and beyond the box; with open ends, the
  value beyond an end plane is eq. inlet's u(x'') - (2 h_z / d) u(x);
* E at a particle is the trilinear interpolation of the nodal E of its cell's corners; a
  particle outside every cell gets E = 0.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import dataclasses
from typing import Tuple

import numpy as np


@dataclasses.dataclass
class Grid:
    dims: Tuple[int, int, int]          # box nx, ny, nz
    z_offset: int                       # box plane of the lattice's plane 0
    origin: Tuple[float, float, float]  # coordinates of lattice node (0, 0, 0)
    h: Tuple[float, float, float]
    robin_d: float = 0.0

    @property
    def lattice(self) -> Tuple[int, int, int]:
        nx, ny, nz = self.dims
        return nx, ny, nz - 2 * self.z_offset


def _cells(g: Grid, pos: np.ndarray):
    """Cell index (i, j, k) of each particle, fractional offsets, and the inside flag."""
    n = np.array(g.lattice)
    u = (pos - np.array(g.origin)) / np.array(g.h)
    c = np.floor(u).astype(np.int64)
    f = u - c
    ok = np.all((c >= 0) & (c <= n - 2), axis=1)
    return c, f, ok


def deposit(g: Grid, pos: np.ndarray, q: float) -> np.ndarray:
    """Charge density on the box, (nz, ny, nx), by cloud-in-cell weights."""
    nx, ny, nz = g.dims
    rho = np.zeros(nx * ny * nz)
    c, f, ok = _cells(g, pos)
    c, f = c[ok], f[ok]
    for dz in (0, 1):
        wz = f[:, 2] if dz else 1.0 - f[:, 2]
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1.0 - f[:, 1]
            for dx in (0, 1):
                wx = f[:, 0] if dx else 1.0 - f[:, 0]
                node = (c[:, 0] + dx) + nx * ((c[:, 1] + dy) + ny * (c[:, 2] + dz + g.z_offset))
                np.add.at(rho, node, q * wx * wy * wz)
    return (rho / (g.h[0] * g.h[1] * g.h[2])).reshape(nz, ny, nx)


def nodal_field(g: Grid, phi: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """E = -grad(phi) at every box node, (3, nz, ny, nx)."""
    nx, ny, nz = g.dims
    p = np.where(mask, phi.reshape(nz, ny, nx), 0.0)
    ext = np.zeros((nz + 2, ny + 2, nx + 2))
    ext[1:-1, 1:-1, 1:-1] = p
    if g.robin_d > 0.0 and g.z_offset == 1:
        # ghost planes beyond the open ends: eq. inlet, u(x') = u(x'') - (2 h / d) u(x)
        r = 2.0 * g.h[2] / g.robin_d
        ext[1, 1:-1, 1:-1] = np.where(mask[1], p[2] - r * p[1], 0.0)
        ext[-2, 1:-1, 1:-1] = np.where(mask[-2], p[-3] - r * p[-2], 0.0)
    E = np.empty((3, nz, ny, nx))
    E[0] = -(ext[1:-1, 1:-1, 2:] - ext[1:-1, 1:-1, :-2]) / (2.0 * g.h[0])
    E[1] = -(ext[1:-1, 2:, 1:-1] - ext[1:-1, :-2, 1:-1]) / (2.0 * g.h[1])
    E[2] = -(ext[2:, 1:-1, 1:-1] - ext[:-2, 1:-1, 1:-1]) / (2.0 * g.h[2])
    return E


def gather(g: Grid, phi: np.ndarray, mask: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """E at the particles, (n, 3)."""
    E = nodal_field(g, phi, mask)
    out = np.zeros((pos.shape[0], 3))
    c, f, ok = _cells(g, pos)
    for dz in (0, 1):
        wz = f[:, 2] if dz else 1.0 - f[:, 2]
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1.0 - f[:, 1]
            for dx in (0, 1):
                wx = f[:, 0] if dx else 1.0 - f[:, 0]
                w = np.where(ok, wx * wy * wz, 0.0)
                i = np.clip(c[:, 0] + dx, 0, g.dims[0] - 1)
                j = np.clip(c[:, 1] + dy, 0, g.dims[1] - 1)
                k = np.clip(c[:, 2] + dz + g.z_offset, 0, g.dims[2] - 1)
                for a in range(3):
                    out[:, a] += w * E[a, k, j, i]
    return out
