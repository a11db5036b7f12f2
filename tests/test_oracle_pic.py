"""Pins of the oracle's cloud-in-cell deposition and field gather (CPU)."""
import numpy as np

import workloads as W
from oracle import grid, pic


def _lattice_grid(shape, nx, ny, nz, robin=False):
    dom = grid.from_shape(shape, nx, ny, nz, robin=robin)
    origin = (-shape.a, -shape.b, -0.5 * shape.length)
    return pic.Grid((dom.nx, dom.ny, dom.nz), int(robin), origin, dom.h, dom.robin_d), dom


def test_single_particle_weights_conserve_charge_and_centroid():
    g, _ = _lattice_grid(W.Shape.cylinder(1.0, 2.0), 11, 11, 9)
    p = np.array([[0.137, -0.271, 0.4115]])
    rho = pic.deposit(g, p, 0.5)
    cell = rho * np.prod(g.h)
    assert abs(cell.sum() - 0.5) < 1e-15 and np.count_nonzero(cell) == 8
    k, j, i = np.nonzero(cell)
    xs = g.origin[0] + i * g.h[0]
    ys = g.origin[1] + j * g.h[1]
    zs = g.origin[2] + (k - g.z_offset) * g.h[2]
    w = cell[k, j, i] / 0.5
    assert np.allclose([w @ xs, w @ ys, w @ zs], p[0], rtol=0, atol=1e-14)


def test_deposit_matches_generator_and_drops_outside_particles():
    shape = W.Shape.ellipse(1.0, 0.6, 4.0)
    g, _ = _lattice_grid(shape, 33, 21, 41)
    pts = W.draw_particles(W.Bunch(5000, (0.3, 0.2, 1.0), seed=11))
    pts = np.vstack([pts, [[5.0, 0.0, 0.0], [0.0, 0.0, -9.0]]])  # two outside the box
    q = 1.0 / len(pts)
    rho = pic.deposit(g, pts, q)
    want = W.cic_deposit(shape, 33, 21, 41, pts)
    assert np.allclose(rho, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    inside = pic._cells(g, pts)[2].sum()
    assert 4000 < inside < 5000  # the bunch spills past the box; those particles are dropped
    assert abs(rho.sum() * np.prod(g.h) - inside * q) < 1e-12


def test_gather_linear_potential_exact():
    """phi = a x + b y + c z: central differences and trilinear weights reproduce -(a, b, c)."""
    shape = W.Shape(W.BOXBORE, 1.0, 0.7, 2.0, 0.1, 2.0)
    g, dom = _lattice_grid(shape, 21, 17, 19)
    nx, ny, nz = g.dims
    x = g.origin[0] + np.arange(nx) * g.h[0]
    y = g.origin[1] + np.arange(ny) * g.h[1]
    z = g.origin[2] + np.arange(nz) * g.h[2]
    phi = 0.3 * x[None, None, :] - 1.7 * y[None, :, None] + 0.9 * z[:, None, None] + 0.25
    rng = np.random.default_rng(5)
    pts = rng.uniform(-0.6, 0.6, size=(400, 3)) * [1.0, 0.7, 1.0]  # away from the faces
    E = pic.gather(g, phi, dom.mask, pts)
    assert np.allclose(E, [-0.3, 1.7, -0.9], rtol=0, atol=1e-12)


def test_gather_open_end_ghost_is_eq_inlet():
    """phi = z^2 - 3 d^2 satisfies the Robin condition, so eq. inlet's ghost value is exact
    and E_z = -2 z at particles right next to the open ends."""
    shape = W.Shape(W.BOXBORE, 1.0, 0.7, 2.0, 0.1, 2.0)
    g, dom = _lattice_grid(shape, 13, 11, 15, robin=True)
    d = 0.5 * shape.length
    nx, ny, nz = g.dims
    z = g.origin[2] + (np.arange(nz) - 1) * g.h[2]
    phi = np.broadcast_to((z * z - 3 * d * d)[:, None, None], (nz, ny, nx)).copy()
    rng = np.random.default_rng(6)
    pts = np.column_stack([rng.uniform(-0.4, 0.4, 200), rng.uniform(-0.3, 0.3, 200),
                           np.concatenate([rng.uniform(-d, -d + 0.2, 100), rng.uniform(d - 0.2, d - 1e-9, 100)])])
    E = pic.gather(g, phi, dom.mask, pts)
    assert np.allclose(E[:, 2], -2.0 * pts[:, 2], rtol=0, atol=1e-12)
    assert np.allclose(E[:, :2], 0.0, atol=1e-12)
