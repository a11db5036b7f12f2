"""Preconditioned conjugate gradients (oracle).

Paper, Section 3.1: the CG algorithm, used unchanged also for the mildly
nonsymmetric matrix of the quadratic wall rule; Section 3.2: preconditioned by one
AMG V-cycle per step; Section 5 (solver comparison): stop when
||r||_2 <= eps ||b||_2.

Readings where the paper leaves a choice open: the residual and right-hand side in the stopping test
are those of the scaled system; beta is the Fletcher-Reeves / Hestenes-Stiefel ratio
(r_new . z_new) / (r . z); when the recursively updated residual passes the test the
true residual b - A x is formed, and the iteration stops only if it passes too,
otherwise it continues from the true residual.  The iteration count is the number
of products with A inside the loop.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE = 0, 4, 5, 6


@dataclasses.dataclass
class Result:
    x: np.ndarray
    iterations: int
    rel_res_true: float
    rel_res_recursive: float
    status: int
    replacements: int = 0


def pcg(A, b: np.ndarray, M: Callable[[np.ndarray], np.ndarray],
        x0: Optional[np.ndarray] = None, tol: float = 1e-8, max_iter: int = 500) -> Result:
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return Result(np.zeros_like(b), 0, 0.0, 0.0, OK)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    rnorm = float(np.linalg.norm(r))
    if rnorm <= tol * bnorm:
        return Result(x, 0, rnorm / bnorm, rnorm / bnorm, OK)
    z = M(r)
    rho = float(np.dot(r, z))
    p = z.copy()
    replacements = 0
    for k in range(1, max_iter + 1):
        q = A @ p
        pq = float(np.dot(p, q))
        if not np.isfinite(pq) or not np.isfinite(rho):
            return Result(x, k, np.nan, np.nan, NONFINITE, replacements)
        if pq <= 0.0 or rho <= 0.0:
            rt = float(np.linalg.norm(b - A @ x)) / bnorm
            return Result(x, k, rt, rnorm / bnorm, BREAKDOWN, replacements)
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rnorm = float(np.linalg.norm(r))
        if rnorm <= tol * bnorm:
            rt = b - A @ x
            rtn = float(np.linalg.norm(rt))
            if rtn <= tol * bnorm:
                return Result(x, k, rtn / bnorm, rnorm / bnorm, OK, replacements)
            r = rt
            rnorm = rtn
            replacements += 1
        z = M(r)
        rho_new = float(np.dot(r, z))
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    rt = float(np.linalg.norm(b - A @ x)) / bnorm
    return Result(x, max_iter, rt, rnorm / bnorm, NOT_CONVERGED, replacements)
