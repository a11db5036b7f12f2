"""Smoothed-aggregation AMG preconditioner (oracle).

Paper, Section 3.2 and Table 1:

* aggregates are cubes of 3^d lattice vertices (prolongation-operator paragraph); the
  tentative prolongator has a 1 in row i, column j when vertex i belongs to aggregate j;
* the tentative prolongator is smoothed by one damped-Jacobi step,
  P = (I - omega D^-1 A) P_tent;
* restriction is the transpose, R = P^T, and the level operator is the Galerkin
  product A_{l+1} = P^T A_l P;
* the smoother is a Chebyshev polynomial in D^-1 A on an interval below an estimate
  of the largest eigenvalue, used for both pre- and post-smoothing;
* the coarsest level (at most ``max_coarse`` = 1000 unknowns) is solved directly;
* the cycle is the V-cycle of Algorithm 1.

Readings where the paper is silent:

* aggregates are the index blocks [3I, 3I+3) x [3J, 3J+3) x [3K, 3K+3) of the level's
  logical box; a block's unknowns form one aggregate, partial blocks are kept; the
  coarse level's logical box has ceil(n/3) points per axis;
* the smoother paragraph asks for a bound on the spectrum without naming a routine.
  lambda_hat is the largest Ritz value of ``eig_iters`` = 15 Lanczos steps on the
  symmetric part S = (A + A^T)/2 in the D inner product (S = A for the symmetric
  variant; for the quadratic rule the largest eigenvalue of D^-1 S bounds the real parts
  of the spectrum of D^-1 A from above).  The start vector holds, at an unknown with
  logical box index i, the SplitMix64 output for counter i (Steele, Lea and Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014) mapped to [-1/2, 1/2);
  the recurrence stops early when beta_k <= 1e-12 * max_j |alpha_j|, and at most n
  steps run on a level with n unknowns;
* omega = (4/3) / lambda_hat; the Chebyshev interval is [lambda_hi / 10, lambda_hi]
  with lambda_hi = 1.1 * lambda_hat, degree 2;
* the Chebyshev recurrence is the classical three-term Chebyshev acceleration
  (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1) preconditioned by D.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


@dataclasses.dataclass
class Options:
    max_coarse: int = 1000
    max_levels: int = 10
    cheb_degree: int = 2
    cheb_ratio: float = 10.0
    cheb_boost: float = 1.1
    eig_iters: int = 15
    omega_scale: float = 4.0 / 3.0
    coarse_solver: str = "direct"   # "direct", or "gs": Gauss-Seidel sweeps (Section 3.2)
    coarse_sweeps: int = 3


@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    D: np.ndarray
    dims: Tuple[int, int, int]        # logical box of this level
    lin: np.ndarray                    # logical box index of each unknown (ascending)
    lam: float = 0.0
    lam_hi: float = 0.0
    omega: float = 0.0
    Ptent: Optional[sp.csr_matrix] = None
    P: Optional[sp.csr_matrix] = None

    @property
    def n(self) -> int:
        return self.lin.size


@dataclasses.dataclass
class Hierarchy:
    levels: List[Level]
    opts: Options
    coarse_lu: tuple = None

    @property
    def sizes(self) -> List[int]:
        return [lv.n for lv in self.levels]


_U64 = np.uint64


def start_vector(lin: np.ndarray) -> np.ndarray:
    """Lanczos start vector: SplitMix64 of the logical box index, as a double in [-1/2, 1/2).

    SplitMix64 value number i: z = (i + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
    z ^= z >> 31.  The top 53 bits scaled by 2^-53 give a value in [0, 1).
    """
    with np.errstate(over="ignore"):
        z = (lin.astype(_U64) + _U64(1)) * _U64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)
        z = z ^ (z >> _U64(31))
    return (z >> _U64(11)).astype(np.float64) / 2.0 ** 53 - 0.5


def lanczos_lambda(A: sp.csr_matrix, D: np.ndarray, lin: np.ndarray, steps: int) -> float:
    """Estimate of the top of the spectrum of D^-1 A by Lanczos on its symmetric part.

    D^-1 S with S = (A + A^T)/2 is self-adjoint in <u, w>_D = u^T D w, so the textbook
    three-term Lanczos recurrence in that inner product builds a tridiagonal T whose
    largest eigenvalue approaches lambda_max(D^-1 S) from below.
    """
    S = ((A + A.T) * 0.5).tocsr()
    dot = lambda u, w: float(np.dot(u, D * w))
    q = start_vector(lin)
    q = q / np.sqrt(dot(q, q))
    q_prev = np.zeros_like(q)
    beta_prev = 0.0
    alpha, beta = [], []
    for _ in range(min(steps, lin.size)):
        w = (S @ q) / D
        a = dot(q, w)
        w = w - a * q - beta_prev * q_prev
        b = np.sqrt(dot(w, w))
        alpha.append(a)
        beta.append(b)
        if b <= 1e-12 * max(abs(x) for x in alpha):
            break
        q_prev, q, beta_prev = q, w / b, b
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


def aggregate(lin: np.ndarray, dims: Tuple[int, int, int]):
    """Aggregate id of each unknown, the coarse unknowns' logical indices and box."""
    mx, my, mz = dims
    X = lin % mx
    Y = (lin // mx) % my
    Z = lin // (mx * my)
    cdims = (-(-mx // 3), -(-my // 3), -(-mz // 3))
    clin = X // 3 + cdims[0] * (Y // 3 + cdims[1] * (Z // 3))
    coarse, agg = np.unique(clin, return_inverse=True)
    return agg.astype(np.int64), coarse.astype(np.int64), cdims


def tentative_prolongator(agg: np.ndarray, nc: int) -> sp.csr_matrix:
    n = agg.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))


def chebyshev(lv: Level, f: np.ndarray, x: Optional[np.ndarray], degree: int,
              ratio: float) -> np.ndarray:
    """Chebyshev smoothing of A x = f on [lam_hi/ratio, lam_hi], preconditioned by D.

    ``x is None`` means a zero initial guess (the pre-smoother of Algorithm 1).
    """
    hi = lv.lam_hi
    lo = hi / ratio
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma1 = theta / delta
    rho = 1.0 / sigma1
    if x is None:
        x = np.zeros_like(f)
        r = f.copy()
    else:
        r = f - lv.A @ x
    d = r / lv.D / theta
    x = x + d
    for _ in range(1, degree):
        r = f - lv.A @ x
        rho_new = 1.0 / (2.0 * sigma1 - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (r / lv.D)
        rho = rho_new
        x = x + d
    return x


def setup(A0: sp.csr_matrix, dims0: Tuple[int, int, int], lin0: np.ndarray,
          opts: Optional[Options] = None) -> Hierarchy:
    """Build the level hierarchy, coarsening until a level has at most max_coarse unknowns."""
    opts = opts or Options()
    A = A0.tocsr()
    levels = [Level(A, A.diagonal().copy(), dims0, lin0)]
    while levels[-1].n > opts.max_coarse and len(levels) < opts.max_levels:
        lv = levels[-1]
        agg, clin, cdims = aggregate(lv.lin, lv.dims)
        if clin.size >= lv.n:
            break
        lv.lam = lanczos_lambda(lv.A, lv.D, lv.lin, opts.eig_iters)
        lv.lam_hi = opts.cheb_boost * lv.lam
        lv.omega = opts.omega_scale / lv.lam
        lv.Ptent = tentative_prolongator(agg, clin.size)
        Dinv = sp.diags(1.0 / lv.D)
        lv.P = (lv.Ptent - lv.omega * (Dinv @ (lv.A @ lv.Ptent))).tocsr()
        Ac = (lv.P.T @ (lv.A @ lv.P)).tocsr()
        Ac.sort_indices()
        levels.append(Level(Ac, Ac.diagonal().copy(), cdims, clin))
    H = Hierarchy(levels, opts)
    H.coarse_lu = sla.lu_factor(levels[-1].A.toarray())
    return H


def refresh(H: Hierarchy, A0: sp.csr_matrix) -> Hierarchy:
    """Reuse of the aggregation hierarchy (Section 5.2): keep every level's logical box,
    unknowns and tentative prolongator from ``H``, and recompute from the new level-0
    operator ``A0`` what depends on the numbers -- the smoother's spectral bound, the
    smoothed prolongators, the Galerkin operators and the coarse solver.

    ``A0`` must act on H's level-0 unknowns (same order).
    """
    old = H.levels
    if A0.shape[0] != old[0].n:
        raise ValueError("the new operator does not act on the hierarchy's unknowns")
    opts = H.opts
    A = A0.tocsr()
    levels = [Level(A, A.diagonal().copy(), old[0].dims, old[0].lin)]
    for k in range(len(old) - 1):
        lv = levels[-1]
        lv.Ptent = old[k].Ptent
        lv.lam = lanczos_lambda(lv.A, lv.D, lv.lin, opts.eig_iters)
        lv.lam_hi = opts.cheb_boost * lv.lam
        lv.omega = opts.omega_scale / lv.lam
        Dinv = sp.diags(1.0 / lv.D)
        lv.P = (lv.Ptent - lv.omega * (Dinv @ (lv.A @ lv.Ptent))).tocsr()
        Ac = (lv.P.T @ (lv.A @ lv.P)).tocsr()
        Ac.sort_indices()
        levels.append(Level(Ac, Ac.diagonal().copy(), old[k + 1].dims, old[k + 1].lin))
    R = Hierarchy(levels, opts)
    R.coarse_lu = sla.lu_factor(levels[-1].A.toarray())
    return R


def gs_colours(lin: np.ndarray, dims: Tuple[int, int, int]) -> np.ndarray:
    """Colour 0..7 of each unknown from the parities of its logical box coordinates."""
    mx, my, _ = dims
    X, Y, Z = lin % mx, (lin // mx) % my, lin // (mx * my)
    return (X & 1) + 2 * (Y & 1) + 4 * (Z & 1)


def gauss_seidel(lv: Level, b: np.ndarray, sweeps: int) -> np.ndarray:
    """Gauss-Seidel sweeps on A x = b from x = 0 (the iterative coarse level solver of
    Section 3.2, three sweeps in the paper).

    Reading: the paper does not fix the ordering.  Unknowns are visited colour by colour
    (colour = parities of the logical coordinates); two unknowns of one colour are never
    coupled by the 27-point coarse stencil, so updating a whole colour at once is exactly
    the sequential sweep in that order.
    """
    col = gs_colours(lv.lin, lv.dims)
    x = np.zeros_like(b)
    for _ in range(sweeps):
        for c in range(8):
            sel = np.nonzero(col == c)[0]
            if sel.size:
                x[sel] += (b[sel] - lv.A[sel] @ x) / lv.D[sel]
    return x


def coarse_solve(H: Hierarchy, b: np.ndarray) -> np.ndarray:
    if H.opts.coarse_solver == "gs" and len(H.levels) > 1:
        return gauss_seidel(H.levels[-1], b, H.opts.coarse_sweeps)
    return sla.lu_solve(H.coarse_lu, b)


def vcycle(H: Hierarchy, b: np.ndarray, level: int = 0) -> np.ndarray:
    """Algorithm 1 (MultiGridSolve) with a zero initial guess on the given level."""
    if level == len(H.levels) - 1:
        return coarse_solve(H, b)
    lv = H.levels[level]
    o = H.opts
    x = chebyshev(lv, b, None, o.cheb_degree, o.cheb_ratio)          # pre-smoothing
    r = b - lv.A @ x                                                   # residual
    bc = lv.P.T @ r                                                    # restriction R = P^T
    v = vcycle(H, bc, level + 1)                                       # coarse problem
    x = x + lv.P @ v                                                   # coarse-grid correction
    return chebyshev(lv, b, x, o.cheb_degree, o.cheb_ratio)           # post-smoothing


def coarse_box_coords(lv: Level) -> np.ndarray:
    """(n, 3) logical (X, Y, Z) coordinates of a level's unknowns."""
    mx, my, _ = lv.dims
    return np.stack([lv.lin % mx, (lv.lin // mx) % my, lv.lin // (mx * my)], axis=1)
