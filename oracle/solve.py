"""End-to-end oracle solve: domain -> scaled system -> SA-AMG hierarchy -> PCG.

Paper, Sections 2 to 4.  The level-0 logical box is the lattice box itself.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Optional

import numpy as np

from . import amg, grid, operator, pcg


@dataclasses.dataclass
class OracleSolve:
    system: operator.System
    hierarchy: amg.Hierarchy
    result: pcg.Result
    x_box: np.ndarray
    t_setup: float
    t_solve: float


def build(shape, nx: int, ny: int, nz: int, variant: int,
          opts: Optional[amg.Options] = None, robin: bool = False):
    """System and hierarchy; with ``robin`` the ends are open and the box has nz + 2 planes."""
    dom = grid.from_shape(shape, nx, ny, nz, robin)
    sys_ = operator.assemble(dom, variant)
    H = amg.setup(sys_.As, (dom.nx, dom.ny, dom.nz), sys_.idx, opts)
    return sys_, H


def refresh(shape, nx: int, ny: int, nz: int, variant: int, H: amg.Hierarchy,
            robin: bool = False):
    """System of a new geometry on the same lattice, and H refreshed for it
    (amg.refresh); the new domain must have H's unknowns."""
    dom = grid.from_shape(shape, nx, ny, nz, robin)
    sys_ = operator.assemble(dom, variant)
    if not np.array_equal(sys_.idx, H.levels[0].lin):
        raise ValueError("the domain's unknowns differ from the hierarchy's")
    return sys_, amg.refresh(H, sys_.As)


def solve(sys_: operator.System, H: amg.Hierarchy, b_box: np.ndarray,
          x0_box: Optional[np.ndarray] = None, tol: float = 1e-8,
          max_iter: int = 500) -> pcg.Result:
    """Solve with unscaled b and x0 on the box; returns the result in scaled variables."""
    bs = operator.scaled_rhs(sys_, b_box)
    y0 = None if x0_box is None else sys_.gather(x0_box) / sys_.sigma
    return pcg.pcg(sys_.As, bs, lambda r: amg.vcycle(H, r), y0, tol, max_iter)


def run(shape, nx, ny, nz, variant, b_box, x0_box=None, tol=1e-8, max_iter=500,
        opts=None, robin: bool = False) -> OracleSolve:
    t0 = time.perf_counter()
    sys_, H = build(shape, nx, ny, nz, variant, opts, robin)
    t1 = time.perf_counter()
    res = solve(sys_, H, b_box, x0_box, tol, max_iter)
    t2 = time.perf_counter()
    x_box = sys_.scatter(operator.unscale(sys_, res.x))
    return OracleSolve(sys_, H, res, x_box, t1 - t0, t2 - t1)
