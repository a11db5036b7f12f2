"""Pins of the oracle's lattice and wall rules against the paper and closed forms (CPU)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import amg, grid, operator, pcg, rows

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _dom(shape, n, nz=None):
    return grid.from_shape(shape, n, n, nz or n)


# --------------------------------------------------------------------------- lattice


def test_paper_dof_counts_cross_section():
    """The tube meshes of the solver-comparison table: all 256 planes times the disc count."""
    g = GOLD["dof_counts"]
    assert grid.cross_section_count(0, 1.0, 1.0, 128, 128) * 256 == g["mesh_128x128x256"]
    assert grid.cross_section_count(0, 1.0, 1.0, 166, 166) * 256 == g["mesh_166x166x256"]


def test_lattice_point_on_the_wall_is_not_an_unknown():
    """On 83 nodes per axis of the unit disc, (9/41, 40/41) lies exactly on r = 1 (a
    Pythagorean triple); it is a wall point, not an unknown, and every neighbouring unknown
    has a positive wall fraction."""
    from fractions import Fraction
    xi, yj = Fraction(2 * 50 - 82, 82), Fraction(2 * 81 - 82, 82)
    assert xi * xi + yj * yj == 1
    dom = grid.from_shape(W.Shape.cylinder(1.0, 6.0), 83, 83, 9)
    assert not dom.mask[4, 81, 50] and not dom.mask[4, 50, 81]
    assert dom.mask[4, 80, 50] and np.all(dom.frac[:, dom.mask] > 0.0)


def test_cylinder33_unknowns():
    w = W.c1_cylinder33()
    assert grid.from_shape(w.shape, 33, 33, 33).n_unknowns == 24583


@pytest.mark.parametrize("shape,n,nz", [
    (W.Shape.cylinder(1.0, 2.0), 21, 17),
    (W.Shape.ellipse(1.0, 0.6, 3.0), 25, 19),
    (W.Shape.boxbore(0.8, 4.0, 0.5), 23, 31),
])
def test_wall_points_lie_on_the_surface(shape, n, nz):
    """x - s h e lands on the implicit wall surface (or on a cap / box face when s = 1)."""
    dom = _dom(shape, n, nz)
    xs = grid.coords(shape.a, n)
    ys = grid.coords(shape.b, n)
    zs = grid.coords(0.5 * shape.length, nz)
    d, k, j, i = np.nonzero(dom.frac < 1.0)
    assert d.size > 0
    s = dom.frac[d, k, j, i]
    assert np.all((s > 0) & (s < 1))
    px, py, pz = xs[i].copy(), ys[j].copy(), zs[k].copy()
    sign = np.where(d % 2 == 0, -1.0, 1.0)
    for ax, p in enumerate((px, py, pz)):
        sel = d // 2 == ax
        p[sel] += sign[sel] * s[sel] * dom.h[ax]
    if shape.kind == W.CYLINDER:
        resid = px ** 2 + py ** 2 - shape.a ** 2
    elif shape.kind == W.ELLIPSE:
        resid = (px / shape.a) ** 2 + (py / shape.b) ** 2 - 1.0
    else:
        on_bore = np.abs(px ** 2 + py ** 2 - shape.bore_r ** 2)
        on_cap = np.abs(np.abs(pz) - shape.cavity_half_len)
        resid = np.minimum(on_bore, on_cap)
    assert np.max(np.abs(resid)) < 1e-12


def test_mask_mirror_symmetry():
    dom = _dom(W.Shape.ellipse(1.0, 0.6, 2.0), 31, 21)
    m = dom.mask
    assert np.array_equal(m, m[:, :, ::-1]) and np.array_equal(m, m[:, ::-1, :])
    assert np.array_equal(m, m[::-1, :, :])
    assert not m[0].any() and not m[-1].any()


# --------------------------------------------------------------------------- operator


def test_linear_rule_symmetric_positive_definite():
    dom = _dom(W.Shape.cylinder(1.0, 2.0), 15)
    s = operator.assemble(dom, operator.LIN)
    A = s.A.toarray()
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)


def test_quadratic_rule_mildly_nonsymmetric_m_matrix():
    """Paper, end of Section 2: an M-matrix, nonsymmetric only at the wall, PD symmetric part."""
    dom = _dom(W.Shape.cylinder(1.0, 2.0), 15)
    s = operator.assemble(dom, operator.QUAD)
    A = s.A.toarray()
    asym = np.abs(A - A.T).max(axis=1)
    near = np.zeros(s.n, dtype=bool)
    fr = dom.frac.reshape(6, -1)[:, s.idx]
    near = (fr < 1.0).any(axis=0)
    # nonsymmetric rows are exactly rows next to the wall or next to such a row
    assert asym.max() > 0
    nbr_of_near = (np.abs(A[:, near]) > 0).any(axis=1)
    assert np.all(asym[~(near | nbr_of_near)] == 0)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0) and np.all(np.diag(A) > 0)
    assert np.all(A.sum(axis=1) >= -1e-9)
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_quadratic_rule_is_shortley_weller_1d():
    """One wall side at distance s h: the x-part of the row equals the nonuniform
    three-point formula -u'' ~ 2/(hl + hr) ((u - u_l)/hl + (u - u_r)/hr) with u_l = 0,
    hl = s h, hr = h (Shortley-Weller)."""
    dom = _dom(W.Shape.cylinder(1.0, 2.0), 21)
    h = dom.h[0]
    checked = 0
    for d in (0, 1):  # walls on the -x and +x side
        k, j, i = np.nonzero(dom.frac[d] < 1.0)
        for kk, jj, ii in zip(k, j, i):
            if dom.frac[1 - d, kk, jj, ii] < 1.0:
                continue
            s = dom.frac[d, kk, jj, ii]
            _, offs, _ = rows.row(dom, operator.QUAD, ii, jj, kk)
            x_off = [o for o in offs if o[0] != 0]
            assert len(x_off) == 1 and x_off[0][0] == (1 if d == 0 else -1)
            hl, hr = s * h, h
            want_diag = 2.0 / (hl + hr) * (1.0 / hl + 1.0 / hr)
            want_off = -2.0 / ((hl + hr) * hr)
            assert abs(_axis_only(dom, ii, jj, kk, axis=0) - want_diag) < 1e-12 * want_diag
            assert abs(x_off[0][3] - want_off) < 1e-12 * abs(want_off)
            checked += 1
    assert checked > 10


def _axis_only(dom, i, j, k, axis):
    """Diagonal contribution of one axis, computed with the quadratic rule."""
    e = [0, 0, 0]
    e[axis] = 1
    in_m = dom.mask[k - e[2], j - e[1], i - e[0]]
    in_p = dom.mask[k + e[2], j + e[1], i + e[0]]
    s = dom.frac[2 * axis, k, j, i]
    t = dom.frac[2 * axis + 1, k, j, i]
    c_self, _, _ = operator._axis_terms(operator.QUAD, np.array([in_m]), np.array([in_p]),
                                        np.array([s]), np.array([t]))
    return float(c_self[0]) / dom.h[axis] ** 2


def test_quadratic_rule_exact_for_axiswise_quadratics():
    """u = (R^2 - x^2 - y^2)(L^2/4 - z^2) vanishes on the whole wall and is quadratic along
    every grid line, so the quadratic extrapolation reproduces -Laplace(u) exactly."""
    R, L = 1.0, 2.0
    dom = grid.from_shape(W.Shape.cylinder(R, L), 19, 19, 15)
    s = operator.assemble(dom, operator.QUAD)
    x = grid.coords(R, 19)
    z = grid.coords(0.5 * L, 15)
    Z, Y, X = np.meshgrid(z, x, x, indexing="ij")
    u = (R * R - X * X - Y * Y) * (0.25 * L * L - Z * Z)
    lap = 4.0 * (0.25 * L * L - Z * Z) + 2.0 * (R * R - X * X - Y * Y)
    Au = s.A @ s.gather(u)
    assert np.max(np.abs(Au - s.gather(lap))) < 1e-9 * np.max(np.abs(lap))


def test_linear_rule_double_wall_row():
    """Both sides outside on one axis: diagonal (1/s + 1/t)/h^2, no off-diagonals."""
    dom = grid.from_shape(W.Shape.cylinder(1.0, 2.0), 9, 9, 9)
    # make a synthetic one-node-wide line: override fractions on a copy
    k, j, i = 4, 4, 4
    dom.mask[:] = False
    dom.mask[k, j, i] = True
    dom.frac[:] = 1.0
    dom.frac[0, k, j, i], dom.frac[1, k, j, i] = 0.3, 0.6
    diag, offs, _ = rows.row(dom, operator.LIN, i, j, k)
    hx = dom.h[0]
    want = (1 / 0.3 + 1 / 0.6) / hx ** 2 + 2 / dom.h[1] ** 2 + 2 / dom.h[2] ** 2
    assert abs(diag - want) < 1e-12 * want and offs == []
    dq, _, _ = rows.row(dom, operator.QUAD, i, j, k)
    wantq = 2 / (0.3 * 0.6) / hx ** 2 + 2 / dom.h[1] ** 2 + 2 / dom.h[2] ** 2
    assert abs(dq - wantq) < 1e-12 * wantq
    s = operator.assemble(dom, operator.QUAD)
    assert abs(s.A[0, 0] - wantq) < 1e-12 * wantq


@pytest.mark.parametrize("robin", [False, True])
def test_rows_match_assembly(robin):
    dom = grid.from_shape(W.Shape.ellipse(1.0, 0.6, 2.0), 17, 17, 13 - 2 * robin, robin=robin)
    for v in (0, 1, 2):
        s = operator.assemble(dom, v)
        xb = W.random_box_vector((17, 17, 13), 3) * dom.mask
        bb = W.random_box_vector((17, 17, 13), 4)
        want = s.sigma * (s.rho * s.gather(bb) - s.A @ s.gather(xb))
        sel = s.idx[::7]
        got = rows.scaled_residual_rows(dom, v, xb, bb, sel)
        assert np.allclose(got, want[::7], rtol=1e-12, atol=1e-12)


def test_scaled_diagonal_is_one():
    dom = _dom(W.Shape.ellipse(1.0, 0.6, 2.0), 17, 13)
    s = operator.assemble(dom, operator.QUAD)
    assert np.max(np.abs(s.As.diagonal() - 1.0)) < 4e-16


def test_all_rules_agree_when_no_wall_is_cut():
    """With every wall fraction 1 the three rules collapse to the Dirichlet 7-point star."""
    dom = _dom(W.Shape.boxbore(0.8, 2.0, 0.5, cavity_half_len=1.0), 11)
    dom.frac[:] = 1.0
    mats = [operator.assemble(dom, v).A for v in (0, 1, 2)]
    assert (mats[0] != mats[1]).nnz == 0 and (mats[0] != mats[2]).nnz == 0


# --------------------------------------------------------------------------- MMS


def _mms(h_inv, variant):
    shape, nx, ny, nz = W.mms_cylinder(h_inv)
    dom = grid.from_shape(shape, nx, ny, nz)
    s = operator.assemble(dom, variant)
    x = grid.coords(0.5, nx)
    z = grid.coords(0.5, nz)
    Z, Y, X = np.meshgrid(z, x, x, indexing="ij")
    r2 = X * X + Y * Y
    rho = -(np.pi ** 2 * r2 - np.pi ** 2 / 4 - 4) * np.sin(np.pi * (Z - 0.5))
    phi = (0.25 - r2) * np.sin(np.pi * (Z - 0.5))
    H = amg.setup(s.As, (nx, ny, nz), s.idx)
    res = pcg.pcg(s.As, operator.scaled_rhs(s, rho), lambda r: amg.vcycle(H, r), tol=1e-12)
    assert res.status == pcg.OK
    e = operator.unscale(s, res.x) - s.gather(phi)
    h = 1.0 / h_inv
    return np.sqrt(h ** 3 * np.sum(e * e)), np.abs(e).max()


@pytest.mark.parametrize("variant,name", [(0, "const"), (1, "lin"), (2, "quad")])
def test_mms_against_paper_tables(variant, name):
    """Errors at h = 1/64 near the paper's Tables 3-5, and the observed rate from 1/32."""
    g = GOLD["mms_errors"][name]
    l2_32, li_32 = _mms(32, variant)
    l2_64, li_64 = _mms(64, variant)
    rate = np.log2(l2_32 / l2_64)
    if variant == 0:
        assert 0.6 < rate < 1.2
    else:
        assert 1.8 < rate < 2.3
    assert 0.75 < l2_64 / g["h64"]["l2"] < 1.33
    assert 0.75 < li_64 / g["h64"]["linf"] < 1.33


def test_diagonal_helper_matches_assembly():
    dom = _dom(W.Shape.ellipse(1.0, 0.6, 2.0), 21, 19)
    for v in (0, 1, 2):
        s = operator.assemble(dom, v)
        idx, dg = operator.diagonal(dom, v)
        assert np.array_equal(idx, s.idx)
        assert np.max(np.abs(dg - s.A.diagonal())) <= 1e-14 * dg.max()


# --------------------------------------------------------------------------- open ends

def test_robin_dof_count_matches_paper_tubes():
    """With open ends every z-plane of the lattice holds unknowns: the solver-comparison
    tubes count 256 full planes."""
    g = GOLD["dof_counts"]
    dom = grid.from_shape(W.Shape.cylinder(1.0, 2.0), 128, 128, 256, robin=True)
    assert dom.nz == 258 and not dom.mask[0].any() and not dom.mask[-1].any()
    assert dom.n_unknowns == g["mesh_128x128x256"]


def _robin_box(n=(9, 8, 11)):
    nx, ny, nz = n
    shape = W.Shape(W.BOXBORE, 1.0, 0.7, 2.0, 0.1, 2.0)  # cavity longer than the pipe
    return grid.from_shape(shape, nx, ny, nz, robin=True), shape


@pytest.mark.parametrize("variant", [operator.CONST, operator.LIN, operator.QUAD])
def test_robin_exact_for_quadratic_profile(variant):
    """u = (a^2 - x^2)(b^2 - y^2)(z^2 - 3 d^2) vanishes on the box walls and satisfies
    du/dn + u/d = 0 on both ends; second differences and the central Robin difference are
    exact for it, so the discrete solution equals u at every unknown."""
    dom, shape = _robin_box()
    s = operator.assemble(dom, variant)
    a, b, d = shape.a, shape.b, 0.5 * shape.length
    x = grid.coords(a, dom.nx)[None, None, :]
    y = grid.coords(b, dom.ny)[None, :, None]
    zc = grid.coords(d, dom.nz - 2)
    z = np.concatenate([[0.0], zc, [0.0]])[:, None, None]
    X2, Y2, Z2 = a * a - x * x, b * b - y * y, z * z - 3 * d * d
    u = X2 * Y2 * Z2
    f = 2 * Y2 * Z2 + 2 * X2 * Z2 - 2 * X2 * Y2
    bs = operator.scaled_rhs(s, f)
    yv = spla.spsolve(s.As.tocsc(), bs)
    xv = operator.unscale(s, yv)
    ue = s.gather(u)
    assert np.max(np.abs(xv - ue)) <= 1e-10 * np.max(np.abs(ue))


def test_robin_rows_symmetric_for_linear_rule():
    dom = grid.from_shape(W.Shape.cylinder(1.0, 2.0), 13, 13, 9, robin=True)
    s = operator.assemble(dom, operator.LIN)
    assert abs(s.A - s.A.T).max() <= 1e-12 * abs(s.A).max()
    assert np.linalg.eigvalsh(s.As.toarray()).min() > 0.0
    q = operator.assemble(dom, operator.QUAD)
    assert abs(q.A - q.A.T).max() > 1e-6 * abs(q.A).max()


def test_robin_end_row_is_eq_inlet_halved():
    """End-plane row of a node with all in-plane neighbours inside:
    (1/2) [ (2 + 2h/d) u - 2 u'' ] / h_z^2 + (1/2) 7-point x,y part."""
    dom, shape = _robin_box((9, 8, 11))
    s = operator.assemble(dom, operator.LIN)
    k, j, i = 1, 4, 4
    n = i + dom.nx * (j + dom.ny * k)
    r = int(np.searchsorted(s.idx, n))
    hx, hy, hz = dom.h
    d = 0.5 * shape.length
    want_diag = 0.5 * ((2 + 2 * hz / d) / hz ** 2 + 2 / hx ** 2 + 2 / hy ** 2)
    assert abs(s.A[r, r] - want_diag) < 1e-12 * want_diag
    r2 = int(np.searchsorted(s.idx, n + dom.nx * dom.ny))
    assert abs(s.A[r, r2] + 1.0 / hz ** 2) < 1e-12 / hz ** 2
    rx = int(np.searchsorted(s.idx, n + 1))
    assert abs(s.A[r, rx] + 0.5 / hx ** 2) < 1e-12 / hx ** 2


@pytest.mark.parametrize("variant", [operator.CONST, operator.LIN, operator.QUAD])
@pytest.mark.parametrize("robin", [False, True])
def test_matrix_free_residual_matches_assembly(variant, robin):
    """The matrix-free scaled residual used at full size equals D^-1/2 (rho b - A x) from the
    assembled matrix, row by row, on an ellipse (cut walls on every axis) with and
    without open ends."""
    dom = grid.from_shape(W.Shape.ellipse(1.0, 0.6, 2.0), 23, 17, 19, robin=robin)
    s = operator.assemble(dom, variant)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((dom.nz, dom.ny, dom.nx)) * dom.mask
    b = rng.standard_normal((dom.nz, dom.ny, dom.nx))
    r, bn = operator.scaled_residual(dom, variant, x, b)
    want = s.sigma * (s.rho * s.gather(b) - s.A @ s.gather(x))
    assert np.abs(r - want).max() <= 1e-12 * np.abs(want).max()
    assert abs(bn - np.linalg.norm(operator.scaled_rhs(s, b))) <= 1e-13 * bn
