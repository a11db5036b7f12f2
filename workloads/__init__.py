"""Seeded synthetic workloads shared by the solver tests, the benchmark and the oracle.

This module only *describes* problems and draws their right-hand sides.  It holds
none of the solver's arithmetic: no grid classification, no wall distances, no
stencil coefficients.  Both the GPU library (through its own domain builder) and
the CPU oracle (through its own geometry code) turn a :class:`Shape` and a grid
size into a discrete domain independently.

Problem family (paper, Section 2 and Section 5): a beam pipe whose cross-section is
a circle, an ellipse, or a rectangular cavity joined to a circular bore, closed by
two planar end caps.  The lattice spans the bounding box of the pipe, nodes at both
ends of every axis included, so ``h = extent / (n - 1)`` per axis.

Right-hand sides (the charge density rho with eps0 = 1 and total charge 1):

* an analytic Gaussian density sampled at the nodes, and
* a seeded Gaussian particle bunch deposited by cloud-in-cell (trilinear) weights
  onto the eight nodes of the cell holding each particle (Section 4: the particle
  layer uses an area-weighting charge assignment).

The solver ignores right-hand-side values at nodes that are not unknowns, so the
generators below fill the whole box.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional, Tuple

import numpy as np

# Shape kinds; the integer codes are also the ones the C interface uses.
CYLINDER = 0
ELLIPSE = 1
BOXBORE = 2
KIND_NAMES = {CYLINDER: "cylinder", ELLIPSE: "ellipse", BOXBORE: "boxbore"}

# Boundary variants (paper, Section 2): constant, linear and quadratic
# extrapolation at the curved wall.  Integer codes match the C interface.
VARIANT_CONST = 0
VARIANT_LIN = 1
VARIANT_QUAD = 2
VARIANT_NAMES = {VARIANT_CONST: "const", VARIANT_LIN: "lin", VARIANT_QUAD: "quad"}

PREC_FP64 = 0
PREC_MIXED = 1


@dataclasses.dataclass(frozen=True)
class Shape:
    """Analytic beam-pipe shape.

    kind     CYLINDER (radius ``a`` = ``b``), ELLIPSE (semi-axes ``a`` along x and
             ``b`` along y) or BOXBORE (square cavity of half-width ``a`` = ``b``
             over ``|z| < cavity_half_len``, united with a coaxial bore of radius
             ``bore_r`` running the full length).
    a, b     half-extent of the bounding box along x and y.
    length   extent along z; the end caps sit at ``z = -length/2`` and ``+length/2``.
    """

    kind: int
    a: float
    b: float
    length: float
    bore_r: float = 0.0
    cavity_half_len: float = 0.0

    @staticmethod
    def cylinder(radius: float, length: float) -> "Shape":
        return Shape(CYLINDER, radius, radius, length)

    @staticmethod
    def ellipse(a: float, b: float, length: float) -> "Shape":
        return Shape(ELLIPSE, a, b, length)

    @staticmethod
    def boxbore(half_width: float, length: float, bore_r: float = 0.5,
                cavity_half_len: Optional[float] = None) -> "Shape":
        if cavity_half_len is None:
            cavity_half_len = length / 6.0
        return Shape(BOXBORE, half_width, half_width, length, bore_r, cavity_half_len)

    @property
    def name(self) -> str:
        return KIND_NAMES[self.kind]


@dataclasses.dataclass(frozen=True)
class Bunch:
    """Gaussian particle bunch: ``n`` particles ~ N(centre, diag(sigma^2))."""

    n: int
    sigma: Tuple[float, float, float]
    seed: int
    centre: Tuple[float, float, float] = (0.0, 0.0, 0.0)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    shape: Shape
    nx: int
    ny: int
    nz: int
    variant: int
    precision: int
    tol: float = 1e-8
    gauss_sigma: Optional[float] = None   # analytic Gaussian density
    bunch: Optional[Bunch] = None         # CIC-deposited particle bunch
    robin: bool = False                   # open ends: the box has a ghost plane per end

    @property
    def dims(self) -> Tuple[int, int, int]:
        """Box of the discrete domain (nx, ny, nz of the lattice, plus 2 planes if open)."""
        return (self.nx, self.ny, self.nz + 2 * int(self.robin))

    @property
    def box_nodes(self) -> int:
        nx, ny, nz = self.dims
        return nx * ny * nz


def spacing(shape: Shape, nx: int, ny: int, nz: int) -> Tuple[float, float, float]:
    """Grid spacing of a lattice that spans the bounding box with n nodes per axis."""
    return (2.0 * shape.a / (nx - 1), 2.0 * shape.b / (ny - 1), shape.length / (nz - 1))


def _axis(half: float, n: int) -> np.ndarray:
    m = 2.0 * np.arange(n, dtype=np.float64) - (n - 1)
    return half * m / (n - 1)


def gaussian_density(shape: Shape, nx: int, ny: int, nz: int, sigma: float) -> np.ndarray:
    """Unit-charge isotropic Gaussian density at every box node, array (nz, ny, nx)."""
    x = _axis(shape.a, nx)
    y = _axis(shape.b, ny)
    z = _axis(0.5 * shape.length, nz)
    r2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
    return (2.0 * math.pi * sigma * sigma) ** -1.5 * np.exp(-r2 / (2.0 * sigma * sigma))


def draw_particles(bunch: Bunch) -> np.ndarray:
    """(n, 3) particle positions, reproducible from the bunch seed."""
    rng = np.random.default_rng(bunch.seed)
    p = rng.normal(size=(bunch.n, 3))
    p *= np.asarray(bunch.sigma, dtype=np.float64)
    p += np.asarray(bunch.centre, dtype=np.float64)
    return p


def cic_deposit(shape: Shape, nx: int, ny: int, nz: int, particles: np.ndarray,
                shift_z: float = 0.0) -> np.ndarray:
    """Cloud-in-cell deposition of unit total charge; returns density (nz, ny, nx).

    Each particle carries charge 1/N and spreads it to the 8 corner nodes of its cell
    with trilinear weights; the density is charge / (hx*hy*hz).  Particles whose cell
    leaves the box are dropped.
    """
    hx, hy, hz = spacing(shape, nx, ny, nz)
    q = 1.0 / particles.shape[0]
    fx = (particles[:, 0] + shape.a) / hx
    fy = (particles[:, 1] + shape.b) / hy
    fz = (particles[:, 2] + shift_z + 0.5 * shape.length) / hz
    ix = np.floor(fx).astype(np.int64)
    iy = np.floor(fy).astype(np.int64)
    iz = np.floor(fz).astype(np.int64)
    keep = (ix >= 0) & (ix < nx - 1) & (iy >= 0) & (iy < ny - 1) & (iz >= 0) & (iz < nz - 1)
    ix, iy, iz = ix[keep], iy[keep], iz[keep]
    wx, wy, wz = fx[keep] - ix, fy[keep] - iy, fz[keep] - iz
    rho = np.zeros(nx * ny * nz, dtype=np.float64)
    for dz in (0, 1):
        w_z = wz if dz else 1.0 - wz
        for dy in (0, 1):
            w_zy = w_z * (wy if dy else 1.0 - wy)
            for dx in (0, 1):
                w = w_zy * (wx if dx else 1.0 - wx)
                lin = (ix + dx) + nx * ((iy + dy) + ny * (iz + dz))
                rho += np.bincount(lin, weights=w, minlength=rho.size)
    rho *= q / (hx * hy * hz)
    return rho.reshape(nz, ny, nx)


def pad_ends(lattice_box: np.ndarray) -> np.ndarray:
    """Lattice array (nz, ny, nx) placed in a box with one empty plane before and after."""
    out = np.zeros((lattice_box.shape[0] + 2,) + lattice_box.shape[1:], dtype=lattice_box.dtype)
    out[1:-1] = lattice_box
    return out


def rhs(w: Workload, shift_z: float = 0.0, particles: Optional[np.ndarray] = None) -> np.ndarray:
    """Right-hand side (charge density) of a workload on its full box, fp64, shaped like
    ``w.dims`` reversed (open-ended workloads get their ghost planes)."""
    if w.gauss_sigma is not None:
        out = gaussian_density(w.shape, w.nx, w.ny, w.nz, w.gauss_sigma)
    elif w.bunch is None:
        raise ValueError("workload has no right-hand-side recipe")
    else:
        if particles is None:
            particles = draw_particles(w.bunch)
        out = cic_deposit(w.shape, w.nx, w.ny, w.nz, particles, shift_z)
    return pad_ends(out) if w.robin else out


# ----------------------------------------------------------------------------------
# Named workloads.  Sizes follow the problem statements they stand for; each
# docstring gives the recipe.
# ----------------------------------------------------------------------------------

def c1_cylinder33() -> Workload:
    """Cylinder R=1, L=2 on 33^3 nodes (h = 1/16), linear wall rule, Gaussian sigma 0.2, fp64."""
    return Workload("cyl33_lin_fp64", Shape.cylinder(1.0, 2.0), 33, 33, 33,
                    VARIANT_LIN, PREC_FP64, gauss_sigma=0.2)


def c2_ellipse128() -> Workload:
    """Ellipse 1.0 x 0.6, L=4 on 128x128x256, quadratic wall rule, 1M-particle bunch, fp64."""
    return Workload("ell128x128x256_quad_fp64", Shape.ellipse(1.0, 0.6, 4.0), 128, 128, 256,
                    VARIANT_QUAD, PREC_FP64, bunch=Bunch(1_000_000, (0.1, 0.1, 0.3), seed=2))


def c3_ellipse256(precision: int = PREC_MIXED, variant: int = VARIANT_QUAD) -> Workload:
    """Ellipse 1.0 x 0.6, L=4 on 256x256x768 (39.1M unknowns), 1M-particle bunch."""
    tag = "mixed" if precision == PREC_MIXED else "fp64"
    vt = VARIANT_NAMES[variant]
    return Workload(f"ell256x256x768_{vt}_{tag}", Shape.ellipse(1.0, 0.6, 4.0), 256, 256, 768,
                    variant, precision, bunch=Bunch(1_000_000, (0.1, 0.1, 0.3), seed=3))


def c5_cylinder192(precision: int = PREC_MIXED) -> Workload:
    """Cylinder R=1, L=8 on 192x192x1024, linear wall rule, 2M-particle bunch (step 0)."""
    tag = "mixed" if precision == PREC_MIXED else "fp64"
    return Workload(f"cyl192x192x1024_lin_{tag}", Shape.cylinder(1.0, 8.0), 192, 192, 1024,
                    VARIANT_LIN, precision,
                    bunch=Bunch(2_000_000, (0.1, 0.1, 0.3), seed=5, centre=(0.0, 0.0, -2.0)))


def pic_shift(step: int) -> float:
    """Rigid z-shift of the moving bunch at PIC step k (0.02 per step)."""
    return 0.02 * step


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    workload: Workload


def serving_shape(kind: int, ratio: int) -> Shape:
    length = 2.0 * ratio
    if kind == CYLINDER:
        return Shape.cylinder(1.0, length)
    if kind == ELLIPSE:
        return Shape.ellipse(1.0, 0.6, length)
    return Shape.boxbore(0.8, length, bore_r=0.5)


def serving_stream(n_requests: int = 256, qps: float = 10.0, seed: int = 4,
                   edge_lo: int = 32, edge_hi: int = 160,
                   precision: int = PREC_MIXED, variant: int = VARIANT_LIN) -> List[Request]:
    """Poisson arrivals of solve requests over random pipe geometries.

    Kind uniform over {cylinder, ellipse, box-with-bore}; cross-section edge uniform
    over the integers [edge_lo, edge_hi]; length ratio uniform over {1, 2, 3, 4} with
    nz = edge * ratio and L = 2 * ratio.  Each request's bunch has sigma =
    0.1, 0.1, 0.3 times the half-extents of its box and seed 1000 + id.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    kinds = rng.integers(0, 3, size=n_requests)
    edges = rng.integers(edge_lo, edge_hi + 1, size=n_requests)
    ratios = rng.integers(1, 5, size=n_requests)
    out = []
    for i in range(n_requests):
        shape = serving_shape(int(kinds[i]), int(ratios[i]))
        e = int(edges[i])
        nz = e * int(ratios[i])
        sig = (0.1 * shape.a, 0.1 * shape.b, 0.3 * 0.5 * shape.length)
        w = Workload(f"req{i}", shape, e, e, nz, variant, precision,
                     bunch=Bunch(100_000, sig, seed=1000 + i))
        out.append(Request(i, float(t[i]), w))
    return out


def mms_cylinder(h_inv: int) -> Tuple[Shape, int, int, int]:
    """Validation problem of Section 5.1: radius 1/2, z in (-1/2, 1/2), spacing 1/h_inv."""
    n = h_inv + 1
    return Shape.cylinder(0.5, 1.0), n, n, n


def by_name(name: str) -> Workload:
    table = {
        "cyl33": c1_cylinder33,
        "ell128": c2_ellipse128,
        "ell256_mixed": lambda: c3_ellipse256(PREC_MIXED),
        "ell256_fp64": lambda: c3_ellipse256(PREC_FP64),
        "ell256_lin_mixed": lambda: c3_ellipse256(PREC_MIXED, VARIANT_LIN),
        "ell256_lin_fp64": lambda: c3_ellipse256(PREC_FP64, VARIANT_LIN),
        "cyl192_mixed": lambda: c5_cylinder192(PREC_MIXED),
        "cyl192_fp64": lambda: c5_cylinder192(PREC_FP64),
    }
    return table[name]()


def small(shape: Shape, nx: int, ny: int, nz: int, variant: int, precision: int = PREC_FP64,
          seed: int = 7, n_particles: int = 20_000, robin: bool = False) -> Workload:
    """Small bunch workload for parity tests (seeded)."""
    sig = (0.15 * shape.a, 0.15 * shape.b, 0.15 * shape.length)
    return Workload(f"small_{shape.name}_{nx}x{ny}x{nz}", shape, nx, ny, nz, variant, precision,
                    bunch=Bunch(n_particles, sig, seed), robin=robin)


def random_box_vector(dims: Tuple[int, int, int], seed: int) -> np.ndarray:
    """Seeded uniform(-1, 1) vector on the full box, (nz, ny, nx) fp64."""
    nx, ny, nz = dims
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(nz, ny, nx))


# ------------------------------------------------------------------ hand-made domains
#
# Discrete domains given directly as a mask and wall fractions (the saamg_domain input),
# for the method's edge cases that no pipe on the configurations' lattices produces.

DIRS = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


@dataclasses.dataclass
class MaskDomain:
    dims: Tuple[int, int, int]           # (nx, ny, nz)
    h: Tuple[float, float, float]
    mask: np.ndarray                     # (nz, ny, nx) bool
    wall_node: np.ndarray                # box-linear index of an unknown
    wall_dir: np.ndarray                 # 0..5 = -x, +x, -y, +y, -z, +z
    wall_s: np.ndarray                   # fraction in (0, 1)


def _wall_entries(mask: np.ndarray, rng: np.random.Generator, lo: float, keep: float):
    """A seeded fraction in [lo, 1) for about ``keep`` of the (unknown, direction) pairs
    whose neighbour is not an unknown; the other pairs get no entry (fraction 1)."""
    nz, ny, nx = mask.shape
    ks, js, is_ = np.nonzero(mask)
    lin = is_ + nx * (js + ny * ks)
    nodes, dirs, fr = [], [], []
    for d, (dx, dy, dz) in enumerate(DIRS):
        sel = np.nonzero(~mask[ks + dz, js + dy, is_ + dx])[0]
        s = rng.uniform(lo, 1.0, sel.size)
        k = rng.uniform(size=sel.size) < keep
        nodes.append(lin[sel][k])
        dirs.append(np.full(int(k.sum()), d, dtype=np.uint8))
        fr.append(s[k])
    order = np.lexsort((np.concatenate(dirs), np.concatenate(nodes)))
    return (np.concatenate(nodes)[order].astype(np.int64), np.concatenate(dirs)[order],
            np.concatenate(fr)[order])


def thin_lines_domain(seed: int = 12) -> MaskDomain:
    """A box cavity, one-node-wide lines along x, y and z, and two isolated nodes, with
    seeded wall fractions: every node of a line has both neighbours outside on the two
    axes across it (and an isolated node on all three)."""
    nx, ny, nz = 30, 28, 26
    m = np.zeros((nz, ny, nx), dtype=bool)
    m[3:12, 3:13, 3:14] = True      # cavity
    m[8, 18, 3:25] = True           # x-line at z = 8, y = 18
    m[17, 3:24, 20] = True          # y-line at z = 17, x = 20
    m[3:23, 22, 8] = True           # z-line at y = 22, x = 8
    m[20, 10, 14] = True            # isolated nodes
    m[22, 5, 25] = True
    node, d, s = _wall_entries(m, np.random.default_rng(seed), 0.05, 0.875)
    return MaskDomain((nx, ny, nz), (0.05, 0.06, 0.07), m, node, d, s)


def cluster_domain() -> MaskDomain:
    """27 separate 3^3 clusters of unknowns, at aggregate blocks 1, 4 and 7 of each axis:
    the first coarsening gives one isolated node per cluster, which no further
    aggregation reduces.  Wall fractions 1 (no entries)."""
    n = 26
    m = np.zeros((n, n, n), dtype=bool)
    for bz in (1, 4, 7):
        for by in (1, 4, 7):
            for bx in (1, 4, 7):
                m[3 * bz:3 * bz + 3, 3 * by:3 * by + 3, 3 * bx:3 * bx + 3] = True
    e = np.zeros(0, dtype=np.int64)
    return MaskDomain((n, n, n), (0.1, 0.1, 0.1), m, e, e.astype(np.uint8), e.astype(np.float64))
