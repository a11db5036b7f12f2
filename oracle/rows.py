"""Single rows of the Poisson operator, one node at a time (oracle).

For grids too large to assemble in a test, this evaluates (A x)_i for chosen unknowns i
directly from the wall rule of Section 2 (eqs. 7pt-star, lin_extrapol,
quad_extrapol, quad_extrapol1), reading the six neighbours and the wall fractions of
each node.  Pure Python, so only for a few thousand rows.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .grid import Domain

CONST, LIN, QUAD = 0, 1, 2


def row(dom: Domain, variant: int, i: int, j: int, k: int):
    """(diag, [(di, dj, dk, coef), ...], rho) of the unscaled row at unknown (i, j, k).

    On an open end (Robin, eq. inlet) the outside z-neighbour is u(x'') - (2 h / d) u(x),
    and the row, already multiplied by rho = 1/2 there, is returned with that factor."""
    diag = 0.0
    offs = []
    rob = dom.robin_d > 0.0 and (k - 1 == 0 or k + 1 == dom.nz - 1)
    for axis in range(3):
        e = [0, 0, 0]
        e[axis] = 1
        m = (i - e[0], j - e[1], k - e[2])
        p = (i + e[0], j + e[1], k + e[2])
        in_m = bool(dom.mask[m[2], m[1], m[0]])
        in_p = bool(dom.mask[p[2], p[1], p[0]])
        s = float(dom.frac[2 * axis, k, j, i])
        t = float(dom.frac[2 * axis + 1, k, j, i])
        ih2 = 1.0 / (dom.h[axis] ** 2)
        if axis == 2 and rob:
            if not (in_m or in_p):
                raise ValueError("an open end needs an unknown z-neighbour")
            diag += (2.0 + 2.0 * dom.h[2] / dom.robin_d) * ih2
            sgn = 1 if in_p else -1
            offs.append((0, 0, sgn, -2.0 * ih2))
            continue
        if in_m and in_p:
            diag += 2.0 * ih2
            offs += [(-e[0], -e[1], -e[2], -ih2), (e[0], e[1], e[2], -ih2)]
            continue
        if variant == CONST:
            diag += 2.0 * ih2
            if in_m:
                offs.append((-e[0], -e[1], -e[2], -ih2))
            if in_p:
                offs.append((e[0], e[1], e[2], -ih2))
        elif variant == LIN:
            diag += (1.0 if in_m else 1.0 / s) * ih2 + (1.0 if in_p else 1.0 / t) * ih2
            if in_m:
                offs.append((-e[0], -e[1], -e[2], -ih2))
            if in_p:
                offs.append((e[0], e[1], e[2], -ih2))
        else:
            if not in_m and not in_p:
                diag += 2.0 / (s * t) * ih2
            elif not in_m:
                diag += 2.0 / s * ih2
                offs.append((e[0], e[1], e[2], -2.0 / (s + 1.0) * ih2))
            else:
                diag += 2.0 / t * ih2
                offs.append((-e[0], -e[1], -e[2], -2.0 / (t + 1.0) * ih2))
    rho = 0.5 if rob else 1.0
    return rho * diag, [(a, b, c, rho * v) for a, b, c, v in offs], rho


def scaled_residual_rows(dom: Domain, variant: int, x_box: np.ndarray, b_box: np.ndarray,
                         nodes: Sequence[int]) -> np.ndarray:
    """D^-1/2 (b - A x) at the given box-linear unknown indices (x, b unscaled)."""
    nx, ny = dom.nx, dom.ny
    xf = x_box.reshape(-1)
    bf = b_box.reshape(-1)
    out = np.empty(len(nodes))
    for t, n in enumerate(nodes):
        i, j, k = n % nx, (n // nx) % ny, n // (nx * ny)
        diag, offs, rho = row(dom, variant, i, j, k)
        ax = diag * xf[n]
        for di, dj, dk, c in offs:
            ax += c * xf[n + di + nx * (dj + ny * dk)]
        out[t] = (rho * bf[n] - ax) / np.sqrt(diag)
    return out
