"""Pins of the oracle's AMG hierarchy, smoother, V-cycle and PCG (CPU).

Each test checks the oracle against something fixed outside it: closed-form spectra of
the box Laplacian, Chebyshev polynomials, the algebra of Galerkin coarse spaces, an
independent CG implementation, or a dense direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import amg, grid, operator, pcg, solve


def _box_system(n=(11, 9, 13), variant=operator.LIN):
    """Rectangular box domain: every wall fraction is 1, Dirichlet Laplacian."""
    nx, ny, nz = n
    # a box cavity longer than the pipe: the domain is the whole box interior
    shape = W.Shape(W.BOXBORE, 1.0, 0.7, 2.0, 0.1, 2.0)
    dom = grid.from_shape(shape, nx, ny, nz)
    assert np.all(dom.frac == 1.0)
    assert dom.n_unknowns == (nx - 2) * (ny - 2) * (nz - 2)
    return dom, operator.assemble(dom, variant)


def _box_mode(dom, kx, ky, kz):
    nx, ny, nz = dom.nx, dom.ny, dom.nz
    i = np.arange(nx)
    j = np.arange(ny)
    k = np.arange(nz)
    v = (np.sin(np.pi * kz * k / (nz - 1))[:, None, None]
         * np.sin(np.pi * ky * j / (ny - 1))[None, :, None]
         * np.sin(np.pi * kx * i / (nx - 1))[None, None, :])
    lam = sum(2.0 / h ** 2 * (1.0 - np.cos(np.pi * kk / (nn - 1)))
              for h, kk, nn in zip(dom.h, (kx, ky, kz), (nx, ny, nz)))
    return v, lam


def test_box_eigenvector_closed_form():
    dom, s = _box_system()
    v, lam = _box_mode(dom, 2, 3, 1)
    vv = s.gather(v)
    assert np.allclose(s.A @ vv, lam * vv, rtol=0, atol=1e-10 * lam)


def test_start_vector_is_splitmix64():
    """Start vector = the published SplitMix64 sequence (state 0), top 53 bits in [-1/2, 1/2)."""
    import json, os
    with open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.json")) as f:
        ref = [int(h, 16) for h in json.load(f)["outputs_hex"]]
    v = amg.start_vector(np.arange(len(ref)))
    assert np.array_equal(v, np.array([(r >> 11) / 2.0 ** 53 - 0.5 for r in ref]))


def test_lanczos_estimate_symmetric_box():
    """Ritz value <= lambda_max (closed form on the box), close after 15 steps, exact at n steps."""
    dom, s = _box_system((15, 13, 17))
    D = s.A.diagonal()
    lam_max = sum(2.0 / h ** 2 * (1.0 + np.cos(np.pi / (n - 1)))
                  for h, n in zip(dom.h, (dom.nx, dom.ny, dom.nz))) / D[0]
    est = amg.lanczos_lambda(s.A, D, s.idx, 15)
    assert est <= lam_max * (1 + 1e-12)
    assert est > 0.97 * lam_max
    dom, s = _box_system((5, 4, 6))
    D = s.A.diagonal()
    lam_max = sum(2.0 / h ** 2 * (1.0 + np.cos(np.pi / (n - 1)))
                  for h, n in zip(dom.h, (dom.nx, dom.ny, dom.nz))) / D[0]
    assert abs(amg.lanczos_lambda(s.A, D, s.idx, 100) - lam_max) < 1e-10 * lam_max


def test_lanczos_estimate_nonsymmetric_uses_symmetric_part():
    """Quadratic rule: at n steps the estimate is lambda_max of D^-1/2 (A + A^T)/2 D^-1/2 (dense),
    which bounds the real parts of the eigenvalues of D^-1 A."""
    dom = grid.from_shape(W.Shape.ellipse(1.0, 0.6, 2.0), 9, 8, 7)
    s = operator.assemble(dom, operator.QUAD)
    A = s.A.toarray()
    assert not np.allclose(A, A.T)
    D = np.diag(A).copy()
    Dh = 1.0 / np.sqrt(D)
    Ssym = Dh[:, None] * (0.5 * (A + A.T)) * Dh[None, :]
    top = np.linalg.eigvalsh(Ssym)[-1]
    est = amg.lanczos_lambda(s.A, D, s.idx, 10 ** 6)
    assert abs(est - top) < 1e-9 * top
    assert est >= np.linalg.eigvals(A / D[:, None]).real.max() - 1e-12


def test_lanczos_keeps_chebyshev_interval_above_spectrum():
    """15 Lanczos steps with the 1.1 boost cover lambda_max(D^-1 A) on every smoothed level."""
    for shape, n, variant in ((W.Shape.cylinder(1.0, 2.0), (43, 43, 43), W.VARIANT_LIN),
                              (W.Shape.ellipse(1.0, 0.6, 4.0), (31, 31, 62), W.VARIANT_QUAD)):
        sys_, H = solve.build(shape, *n, variant, amg.Options())
        for lv in H.levels[:-1]:
            M = (lv.A.multiply(1.0 / lv.D[:, None])).tocsr()
            top = spla.eigs(M, k=1, which="LR", return_eigenvectors=False, tol=1e-10).real[0]
            assert lv.lam_hi >= 1.05 * top


def test_no_breakdown_cylinder_103():
    """Regression: a 103^3 cylinder (linear rule) whose spectrum a 15-step power estimate from a
    Weyl-sequence start vector placed 21% too low, so PCG broke down; it now converges."""
    req = W.serving_stream(n_requests=48, qps=1.0, seed=4)[18]
    w = req.workload
    assert (w.nx, w.ny, w.nz, w.variant) == (103, 103, 103, W.VARIANT_LIN)
    sys_, H = solve.build(w.shape, w.nx, w.ny, w.nz, w.variant, amg.Options())
    res = solve.solve(sys_, H, W.rhs(w).reshape(-1), None, 1e-8, 100)
    assert res.status == 0 and res.iterations < 20


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_chebyshev_error_polynomial(degree):
    """On an eigenvector of D^-1 A the smoother's error is T_m((theta - mu)/delta) / T_m(theta/delta)."""
    dom, s = _box_system()
    D = s.A.diagonal()
    lv = amg.Level(s.A, D, (dom.nx, dom.ny, dom.nz), s.idx)
    lv.lam_hi = 2.05
    ratio = 30.0
    lo = lv.lam_hi / ratio
    theta, delta = 0.5 * (lv.lam_hi + lo), 0.5 * (lv.lam_hi - lo)
    for mode in ((1, 1, 1), (3, 2, 5), (8, 6, 10)):
        v, lam = _box_mode(dom, *mode)
        e0 = s.gather(v)
        mu = lam / D[0]
        # solve A x = 0 from x0 = e0: the iterate is the propagated error
        e = amg.chebyshev(lv, np.zeros_like(e0), e0, degree, ratio)
        T = np.polynomial.chebyshev.Chebyshev.basis(degree)
        want = T((theta - mu) / delta) / T(theta / delta)
        assert np.allclose(e, want * e0, atol=1e-12 * np.abs(e0).max())


def test_zero_guess_chebyshev_equals_nonzero_form():
    dom, s = _box_system()
    lv = amg.Level(s.A, s.A.diagonal(), (dom.nx, dom.ny, dom.nz), s.idx)
    lv.lam_hi = 2.0
    f = s.gather(W.random_box_vector((dom.nx, dom.ny, dom.nz), 1))
    a = amg.chebyshev(lv, f, None, 2, 30.0)
    b = amg.chebyshev(lv, f, np.zeros_like(f), 2, 30.0)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-14)


def _c1_hier(variant=operator.LIN):
    w = W.c1_cylinder33()
    return solve.build(w.shape, 33, 33, 33, variant)


def test_cylinder33_three_levels():
    """Table 1's coarse-size limit of 1000 gives three levels on the 33^3 cylinder."""
    _, H = _c1_hier()
    assert H.sizes == [24583, 1111, 64]


def test_aggregates_are_3_cubes():
    _, H = _c1_hier()
    lv = H.levels[0]
    cols = lv.Ptent.tocsr().indices
    fine = amg.coarse_box_coords(lv)
    coarse = amg.coarse_box_coords(H.levels[1])
    assert np.array_equal(fine // 3, coarse[cols])
    counts = np.bincount(cols)
    assert counts.max() == 27 and counts.min() >= 1


@pytest.mark.parametrize("variant", [operator.LIN, operator.QUAD])
def test_coarse_operators_are_27_point(variant):
    _, H = _c1_hier(variant)
    for l in (1, 2):
        lv = H.levels[l]
        c = amg.coarse_box_coords(lv)
        A = lv.A.tocoo()
        d = np.abs(c[A.row] - c[A.col]).max(axis=1)
        assert d.max() == 1
        assert np.all(lv.A.diagonal() > 0)


def test_galerkin_two_level_projection():
    """E = I - P (P^T A P)^-1 P^T A is an A-orthogonal projector: E^2 = E, P^T A E = 0."""
    s, H = solve.build(W.Shape.cylinder(1.0, 2.0), 13, 13, 13, operator.LIN,
                       amg.Options(max_coarse=10))
    lv = H.levels[0]
    A = lv.A.toarray()
    P = lv.P.toarray()
    Ac = H.levels[1].A.toarray()
    E = np.eye(A.shape[0]) - P @ np.linalg.solve(Ac, P.T @ A)
    assert np.abs(E @ E - E).max() < 1e-10
    assert np.abs(P.T @ A @ E).max() < 1e-10
    assert np.abs(A @ E - (A @ E).T).max() < 1e-10


# ------------------------------------------------------------------ smoothed prolongator
#
# Section 3.2 smooths the tentative prolongator by one damped-Jacobi step,
# P = (I - omega D^-1 A) P_tent, with omega = (4/3) / lambda_hat.  The three pins below fix
# the damping factor, the sign and the diagonal scaling from outside the oracle's formula:
# a closed form on a box, the energy decrease that damped Jacobi guarantees, and the
# covariance of the whole construction under a diagonal change of variables.


def test_smoothed_prolongator_closed_form_on_box():
    """Box domain, scaled operator (unit diagonal, interior off-diagonals -c_a with
    c_a = sigma^2 / h_a^2 and sum of the six equal to 1), full-length Lanczos so that
    lambda_hat is the closed-form top eigenvalue sum_a 2 c_a (1 + cos(pi / (n_a - 1))).
    Row i of aggregate J: P[i, J] = 1 - omega * (sum of c over the directions whose
    neighbour is not in J, walls included), P[i, J'] = omega * (sum of c over the
    directions whose neighbour is an unknown of J'), every other entry 0."""
    nx, ny, nz = 11, 9, 13
    dom, s = _box_system((nx, ny, nz))
    H = amg.setup(s.As, (nx, ny, nz), s.idx, amg.Options(eig_iters=10 ** 6, max_coarse=10))
    lv = H.levels[0]
    inv_h2 = [1.0 / h ** 2 for h in dom.h]
    c = [v / (2.0 * sum(inv_h2)) for v in inv_h2]
    lam = sum(2.0 * ca * (1.0 + np.cos(np.pi / (n - 1))) for ca, n in zip(c, (nx, ny, nz)))
    omega = (4.0 / 3.0) / lam
    assert abs(lv.omega - omega) <= 1e-12 * omega
    # coarse column of each aggregate block, from the coarse level's logical indices
    cx, cy, cz = H.levels[1].dims
    col_of = {int(q): j for j, q in enumerate(H.levels[1].lin)}
    want = np.zeros(lv.P.shape)
    for row, lin in enumerate(s.idx):
        i, j, k = lin % nx, (lin // nx) % ny, lin // (nx * ny)
        J = col_of[i // 3 + cx * (j // 3 + cy * (k // 3))]
        want[row, J] = 1.0
        for a, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            for sgn in (-1, 1):
                ii, jj, kk = i + sgn * di, j + sgn * dj, k + sgn * dk
                inside = 1 <= ii <= nx - 2 and 1 <= jj <= ny - 2 and 1 <= kk <= nz - 2
                Jn = col_of[ii // 3 + cx * (jj // 3 + cy * (kk // 3))] if inside else None
                if Jn == J:
                    continue
                want[row, J] -= omega * c[a]
                if inside:
                    want[row, Jn] += omega * c[a]
    assert np.abs(lv.P.toarray() - want).max() <= 1e-13


def test_smoothed_prolongator_lowers_column_energy():
    """Damped Jacobi with 0 < omega lambda_max(D^-1 A) < 2 strictly lowers the A-energy of
    every column of the tentative prolongator (linear rule, levels 0 and 1 of the 33^3
    cylinder), and omega lambda_max, with lambda_max from an eigensolver, lies in
    [4/3, 4/3 * 1.015]: lambda_hat is a lower bound within 1.5%."""
    _, H = _c1_hier(operator.LIN)
    for l in (0, 1):
        lv = H.levels[l]
        Dh = sp.diags(1.0 / np.sqrt(lv.D))
        top = spla.eigsh((Dh @ lv.A @ Dh).tocsr(), k=1, which="LA", tol=1e-12,
                         return_eigenvectors=False)[0]
        assert 4.0 / 3.0 * (1 - 1e-12) <= lv.omega * top <= 4.0 / 3.0 * 1.015, (l, lv.omega * top)
        e_tent = (lv.Ptent.T @ (lv.A @ lv.Ptent)).diagonal()
        e_smooth = (lv.P.T @ (lv.A @ lv.P)).diagonal()
        assert np.all(e_smooth < e_tent), l
        assert np.median(e_smooth / e_tent) < 0.9


@pytest.mark.parametrize("variant", [operator.LIN, operator.QUAD])
def test_hierarchy_covariant_under_blockwise_diagonal_scaling(variant):
    """D^-1 A, its spectrum and the Galerkin product are covariant under A -> S A S for a
    positive diagonal S.  When S is constant on each 9^3 block of the lattice (so on every
    aggregate of levels 0 and 1), the setup of S A S must give
        P_0' = S^-1 P_0 S_1,  A_1' = S_1 A_1 S_1,  P_1' = S_1^-1 P_1 S_2,  A_2' = S_2 A_2 S_2,
    with S_l the block value at each level-l unknown.  Dropping D^-1 from the prolongator
    smoothing on any of these levels breaks this."""
    sys_, H = solve.build(W.Shape.cylinder(1.0, 2.0), 23, 23, 21, variant,
                          amg.Options(eig_iters=10 ** 6, max_coarse=20))
    assert len(H.levels) >= 3
    nx, ny, nz = H.levels[0].dims
    blk = np.random.default_rng(5).uniform(0.3, 3.0, (-(-nz // 9), -(-ny // 9), -(-nx // 9)))

    def block_value(l):
        lv = H.levels[l]
        X, Y, Z = amg.coarse_box_coords(lv).T
        f = 9 // 3 ** l
        return blk[Z // f, Y // f, X // f]

    S = [block_value(l) for l in range(3)]
    A0 = (sp.diags(S[0]) @ sys_.As @ sp.diags(S[0])).tocsr()
    G = amg.setup(A0, H.levels[0].dims, H.levels[0].lin, H.opts)
    assert G.sizes == H.sizes
    for l in (0, 1):
        a, b = G.levels[l], H.levels[l]
        assert abs(a.lam - b.lam) <= 1e-11 * b.lam
        want = sp.diags(1.0 / S[l]) @ b.P @ sp.diags(S[l + 1])
        assert abs(a.P - want).max() <= 1e-12 * abs(want).max(), l
        Ac = sp.diags(S[l + 1]) @ H.levels[l + 1].A @ sp.diags(S[l + 1])
        assert abs(G.levels[l + 1].A - Ac).max() <= 1e-11 * abs(Ac).max(), l


def test_vcycle_symmetric_positive_for_linear_rule():
    s, H = _c1_hier(operator.LIN)
    rng = np.random.default_rng(0)
    u, w = rng.standard_normal((2, s.n))
    Mu, Mw = amg.vcycle(H, u), amg.vcycle(H, w)
    assert abs(u @ Mw - w @ Mu) < 1e-12 * abs(u @ Mw)
    assert u @ Mu > 0 and w @ Mw > 0


def test_vcycle_is_linear():
    s, H = _c1_hier(operator.QUAD)
    rng = np.random.default_rng(1)
    u, w = rng.standard_normal((2, s.n))
    lhs = amg.vcycle(H, 2.0 * u - 3.0 * w)
    rhs = 2.0 * amg.vcycle(H, u) - 3.0 * amg.vcycle(H, w)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())


def test_cg_without_preconditioner_matches_scipy():
    s, _ = _c1_hier(operator.LIN)
    b = s.sigma * s.gather(W.rhs(W.c1_cylinder33()))
    res = pcg.pcg(s.As, b, lambda r: r, tol=1e-10, max_iter=2000)
    x_sp, info = spla.cg(s.As, b, rtol=1e-12, maxiter=5000)
    assert res.status == pcg.OK and info == 0
    assert np.linalg.norm(res.x - x_sp) / np.linalg.norm(x_sp) < 1e-8


@pytest.mark.parametrize("variant", [operator.LIN, operator.QUAD, operator.CONST])
def test_pcg_matches_dense_direct_solve(variant):
    shape = W.Shape.ellipse(1.0, 0.6, 2.0)
    wl = W.small(shape, 21, 17, 19, variant)
    s, H = solve.build(shape, 21, 17, 19, variant, amg.Options(max_coarse=100))
    assert len(H.levels) >= 2
    b = W.rhs(wl)
    res = solve.solve(s, H, b, tol=1e-12)
    xd = np.linalg.solve(s.A.toarray(), s.gather(b))
    x = operator.unscale(s, res.x)
    assert res.status == pcg.OK
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9


def test_pcg_box_sine_mode_closed_form():
    """Right-hand side = one eigenvector of the box Laplacian: x = b / lambda."""
    dom, s = _box_system((17, 15, 13))
    v, lam = _box_mode(dom, 1, 2, 1)
    H = amg.setup(s.As, (dom.nx, dom.ny, dom.nz), s.idx, amg.Options(max_coarse=50))
    res = solve.solve(s, H, v, tol=1e-12)
    x = operator.unscale(s, res.x)
    assert np.linalg.norm(x - s.gather(v) / lam) < 1e-9 * np.linalg.norm(s.gather(v) / lam)


def test_pcg_special_cases():
    s, H = _c1_hier(operator.LIN)
    zero = np.zeros((33, 33, 33))
    r0 = solve.solve(s, H, zero)
    assert r0.iterations == 0 and np.all(r0.x == 0)
    b = W.rhs(W.c1_cylinder33())
    full = solve.solve(s, H, b)
    x_box = s.scatter(operator.unscale(s, full.x))
    again = solve.solve(s, H, b, x0_box=x_box)
    assert again.iterations == 0
    near = solve.solve(s, H, b, x0_box=x_box * (1 + 1e-5))
    assert 0 < near.iterations < full.iterations
    one = solve.solve(s, H, b, max_iter=1)
    assert one.status == pcg.NOT_CONVERGED and one.iterations == 1


def test_scaling_leaves_unscaled_solution_unchanged():
    s, H = _c1_hier(operator.QUAD)
    b = W.rhs(W.c1_cylinder33())
    res = solve.solve(s, H, b, tol=1e-12)
    x = operator.unscale(s, res.x)
    r = s.gather(b) - s.A @ x
    assert np.linalg.norm(r) < 1e-9 * np.linalg.norm(s.gather(b))


@pytest.mark.parametrize("variant", [W.VARIANT_LIN, W.VARIANT_QUAD])
def test_pcg_robin_matches_direct_solve(variant):
    """Open ends: the AMG-PCG solution equals a sparse direct solve of the same system."""
    shape = W.Shape.cylinder(1.0, 2.0)
    sys_, H = solve.build(shape, 21, 21, 17, variant, amg.Options(), robin=True)
    assert sys_.dom.nz == 19
    b = W.rhs(W.small(shape, 21, 21, 17, variant, robin=True))
    assert b.shape == (19, 21, 21)
    res = solve.solve(sys_, H, b, tol=1e-12)
    assert res.status == 0
    y = spla.spsolve(sys_.As.tocsc(), operator.scaled_rhs(sys_, b))
    assert np.linalg.norm(res.x - y) <= 1e-9 * np.linalg.norm(y)


def test_colored_gauss_seidel_is_sequential_gauss_seidel():
    """The colour-by-colour sweep equals the textbook sweep x <- (D + L)^-1 (b - U x) in the
    same order (a triangular solve of the permuted matrix)."""
    import scipy.sparse as sp
    shape = W.Shape.ellipse(1.0, 0.6, 4.0)
    sys_, H = solve.build(shape, 45, 30, 60, W.VARIANT_QUAD, amg.Options())
    lv = H.levels[-1]
    assert 27 >= np.diff(lv.A.indptr).max() > 7 and lv.n > 50
    b = np.random.default_rng(3).standard_normal(lv.n)
    order = np.argsort(amg.gs_colours(lv.lin, lv.dims), kind="stable")
    Ap = lv.A[order][:, order].tocsr()
    L = sp.tril(Ap, format="csr")
    U = sp.triu(Ap, k=1, format="csr")
    x = np.zeros(lv.n)
    for _ in range(3):
        x = spla.spsolve_triangular(L, b[order] - U @ x, lower=True)
    want = np.empty(lv.n)
    want[order] = x
    got = amg.gauss_seidel(lv, b, 3)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_pcg_with_gauss_seidel_coarse_solver_converges():
    shape = W.Shape.cylinder(1.0, 2.0)
    for variant in (W.VARIANT_LIN, W.VARIANT_QUAD):
        o = amg.Options(coarse_solver="gs")
        sys_, H = solve.build(shape, 33, 33, 33, variant, o)
        b = W.rhs(W.small(shape, 33, 33, 33, variant))
        res = solve.solve(sys_, H, b, tol=1e-10)
        ref = solve.solve(*solve.build(shape, 33, 33, 33, variant), b, tol=1e-10)
        assert res.status == 0 and res.iterations <= ref.iterations + 3
        assert np.linalg.norm(res.x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


# ------------------------------------------------------------------ hierarchy reuse


@pytest.mark.parametrize("variant,shape1,shape2", [
    # a bunch that elongates: same lattice and unknowns, larger h_z
    (W.VARIANT_LIN, W.Shape.cylinder(1.0, 2.0), W.Shape.cylinder(1.0, 2.6)),
    # a flatter ellipse: the lattice spans the bounding box, so only h_y changes
    (W.VARIANT_QUAD, W.Shape.ellipse(1.0, 0.6, 4.0), W.Shape.ellipse(1.0, 0.45, 4.0)),
])
def test_refresh_equals_fresh_setup(variant, shape1, shape2):
    """Reuse of the aggregation hierarchy (Section 5.2): the aggregates depend on the
    unknowns only, so refreshing a hierarchy for a new geometry with the same unknowns
    gives, level by level, the hierarchy that a fresh setup builds; the numbers do change."""
    n = (33, 29, 31)
    _, H1 = solve.build(shape1, *n, variant)
    s2, R = solve.refresh(shape2, *n, variant, H1)
    _, F = solve.build(shape2, *n, variant)
    assert R.sizes == F.sizes == H1.sizes
    for a, b, old in zip(R.levels, F.levels, H1.levels):
        scale = abs(b.A).max()
        assert abs(a.A - b.A).max() <= 1e-15 * scale
        assert abs(a.A - old.A).max() > 1e-6 * scale
        if b.P is not None:
            assert abs(a.lam - b.lam) <= 1e-15 * b.lam and a.lam != old.lam
            assert abs(a.P - b.P).max() <= 1e-15 * abs(b.P).max()
    r = np.random.default_rng(3).standard_normal(s2.n)
    zr, zf = amg.vcycle(R, r), amg.vcycle(F, r)
    assert np.abs(zr - zf).max() <= 1e-13 * np.abs(zf).max()


def test_refresh_rejects_other_unknowns():
    # the bore radius relative to the cavity changes which lattice nodes are inside
    _, H = solve.build(W.Shape.boxbore(0.8, 4.0, 0.5), 31, 31, 45, W.VARIANT_LIN)
    with pytest.raises(ValueError):
        solve.refresh(W.Shape.boxbore(0.8, 4.0, 0.4), 31, 31, 45, W.VARIANT_LIN, H)


def test_elongating_cylinder_keeps_its_unknowns():
    """The workload of the hierarchy reuse: the lattice spans the bounding box and the
    cylinder does not vary along z, so every length gives the same unknowns and wall
    fractions (only h_z changes)."""
    ref = grid.from_shape(W.Shape.cylinder(1.0, 2.0), 25, 25, 19)
    for L in (2.2, 3.0, 7.5):
        d = grid.from_shape(W.Shape.cylinder(1.0, L), 25, 25, 19)
        assert np.array_equal(d.mask, ref.mask)
        assert np.array_equal(d.frac, ref.frac)
        assert d.h[2] == pytest.approx(L / 18) and d.h[0] == ref.h[0]
