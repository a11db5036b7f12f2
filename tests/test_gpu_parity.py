"""GPU parity: every step of the HIP path against the CPU oracle, through the C-ABI.

Tolerances:
* fp64 components (operator, Galerkin coefficients, smoother, transfers, V-cycle):
  1e-12 relative (only the summation order differs, over at most a few hundred terms
  of bounded size);
* fp64 PCG solution: 1e-8 relative to the oracle's solution of the same algorithm, and
  the same iteration count +-1;
* mixed precision (fp32 hierarchy and V-cycle): single products and transfers 2e-5,
  the two-step smoother and the V-cycle 1e-4 (fp32 unit roundoff 6e-8 times a few dozen
  bounded terms per output, carried through a few chained products and every level),
  full solve 1e-6 relative to the oracle's solution driven to 1e-13.

Component checks are element by element: max |got - want| over max |want|.
"""
import numpy as np
import pytest

import workloads as W
from oracle import amg, grid, operator, pcg, rows, solve

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")

pytestmark = pytest.mark.gpu

CASES = {
    # name: (shape, nx, ny, nz, variant)
    "cyl33_lin": (W.Shape.cylinder(1.0, 2.0), 33, 33, 33, W.VARIANT_LIN),
    "ell70_quad": (W.Shape.ellipse(1.0, 0.6, 4.0), 70, 45, 66, W.VARIANT_QUAD),
    "boxbore_lin": (W.Shape.boxbore(0.8, 4.0, 0.5), 41, 41, 83, W.VARIANT_LIN),
    "cyl_const": (W.Shape.cylinder(1.0, 2.0), 29, 29, 35, W.VARIANT_CONST),
    # open (Robin) ends: lattice nz planes, box nz + 2
    "cyl_robin_lin": (W.Shape.cylinder(1.0, 2.0), 27, 27, 25, W.VARIANT_LIN, True),
    "ell_robin_quad": (W.Shape.ellipse(1.0, 0.6, 4.0), 40, 26, 44, W.VARIANT_QUAD, True),
    "ell68_quad": (W.Shape.ellipse(1.0, 0.6, 4.0), 68, 45, 66, W.VARIANT_QUAD),
    # a symmetric (linear) rule with nx a multiple of 4, for the 16-byte-lane layout
    "cyl36_lin": (W.Shape.cylinder(1.0, 2.0), 36, 36, 40, W.VARIANT_LIN),
}
# (case, lanes): every case with the automatic level-0 lanes (one node per lane on these
# short lines), and the cases whose nx is a multiple of 4 again on 16-byte lanes
# (l0_wide = 2: 4 fp32 / 2 fp64 nodes per lane, lines far shorter than a wavefront's span)
LANES = [(n, 0) for n in CASES] + [(n, 2) for n in CASES if CASES[n][1] % 4 == 0]


def _dev():
    return torch.device("cuda:0")


class Case:
    def __init__(self, name, precision=W.PREC_FP64, opts=None, gs=False, wide=0, ring=0):
        shape, nx, ny, nz, variant = CASES[name][:5]
        robin = len(CASES[name]) > 5 and CASES[name][5]
        self.name, self.shape, self.variant = name, shape, variant
        self.dims = (nx, ny, nz + 2 * int(robin))  # box
        self.precision = precision
        print(f"[case] {name} {nx}x{ny}x{nz} variant={variant} robin={robin} prec={precision} "
              f"wide={wide}", flush=True)
        if gs:
            opts = amg.Options(coarse_solver="gs")
        self.sys, self.H = solve.build(shape, nx, ny, nz, variant, opts, robin=robin)
        dom = sa.domain_for(shape, nx, ny, nz, open_ends=robin)
        o = sa.default_options(precision=precision, l0_wide=wide, cg_ring=ring)
        if opts is not None:
            o.max_coarse, o.cheb_degree = opts.max_coarse, opts.cheb_degree
            o.coarse_solver = sa.COARSE_GS if opts.coarse_solver == "gs" else sa.COARSE_DIRECT
            o.coarse_sweeps = opts.coarse_sweeps
        self.G = sa.setup(dom, variant, o)
        self.info = sa.hierarchy_info(self.G)
        if wide:
            assert self.info["l0_wide"] == int(wide == 2)
        self.b = W.rhs(W.small(shape, nx, ny, nz, variant, robin=robin))

    def to_dev(self, box):
        return torch.from_numpy(np.ascontiguousarray(box, dtype=np.float64).reshape(-1)).to(_dev())

    def lv_box(self, l, v):
        lv = self.H.levels[l]
        mx, my, mz = lv.dims
        out = np.zeros(mx * my * mz)
        out[lv.lin] = v
        return out.reshape(mz, my, mx)

    def lv_vec(self, l, box):
        return box.reshape(-1)[self.H.levels[l].lin]


_cache = {}


def case(name, precision=W.PREC_FP64, gs=False, wide=0, ring=0):
    key = (name, precision, gs, wide, ring)
    if key not in _cache:
        _cache[key] = Case(name, precision, gs=gs, wide=wide, ring=ring)
    return _cache[key]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def emax(a, b):
    """Element-wise error: max |a - b| over max |b|."""
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def oracle_coef(lv):
    mx, my, mz = lv.dims
    c = amg.coarse_box_coords(lv)
    A = lv.A.tocoo()
    d = c[A.col] - c[A.row]
    k = (d[:, 0] + 1) + 3 * (d[:, 1] + 1) + 9 * (d[:, 2] + 1)
    out = np.zeros((27, mz, my, mx))
    out[k, c[A.row, 2], c[A.row, 1], c[A.row, 0]] = A.data
    return out


# ------------------------------------------------------------------ hierarchy


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_matches_oracle(name):
    c = case(name)
    sizes = c.H.sizes
    assert c.info["n_levels"] == len(sizes)
    assert c.info["n_unknowns"] == sizes
    for l, lv in enumerate(c.H.levels):
        assert tuple(c.info["dims"][l]) == tuple(lv.dims)
        if l < len(sizes) - 1:
            assert abs(c.info["lambda_est"][l] - lv.lam) <= 1e-10 * lv.lam
            assert abs(c.info["omega"][l] - lv.omega) <= 1e-10 * lv.omega


@pytest.mark.parametrize("name", [n for n, w in LANES if w == 2])
def test_spectral_estimates_on_wide_lanes(name):
    """Level 0 on 16-byte lanes runs the Lanczos steps' symmetric-part apply on the wide
    march (rows of A and A^T from the table at irregular nodes): the estimates and the
    smoothing weights agree with the oracle's as on one-node lanes."""
    c = case(name, wide=2)
    for l, lv in enumerate(c.H.levels[:-1]):
        assert abs(c.info["lambda_est"][l] - lv.lam) <= 1e-10 * lv.lam, (name, l)
        assert abs(c.info["omega"][l] - lv.omega) <= 1e-10 * lv.omega, (name, l)


@pytest.mark.parametrize("name", list(CASES))
def test_operator_coefficients_every_level(name):
    c = case(name)
    for l, lv in enumerate(c.H.levels):
        got = sa.level_coefficients(c.G, l, lv.dims)
        want = oracle_coef(lv)
        scale = np.abs(want).max()
        tol = 1e-14 if l == 0 else 1e-12
        assert np.abs(got - want).max() <= tol * scale, (name, l)


def test_scaling_vector():
    c = case("ell70_quad")
    sig = torch.zeros(np.prod(c.dims), dtype=torch.float64, device=_dev())
    sa.scaling(c.G, sig)
    want = c.sys.scatter(c.sys.sigma).reshape(-1)
    assert np.abs(sig.cpu().numpy() - want).max() <= 1e-15 * want.max()


# ------------------------------------------------------------------ components


@pytest.mark.parametrize("name,wide", LANES)
@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_level_operations(name, wide, precision):
    c = case(name, precision, wide=wide)
    fp64 = precision == W.PREC_FP64
    tol = 1e-12 if fp64 else 2e-5
    tol_smooth = 1e-12 if fp64 else 1e-4
    rng = np.random.default_rng(11)
    nl = len(c.H.levels)
    for l in range(nl):
        lv = c.H.levels[l]
        mx, my, mz = lv.dims
        x = rng.uniform(-1, 1, lv.n)
        xb = c.lv_box(l, x)
        for op, want in ((sa.capi.OP_APPLY, lv.A @ x), (sa.capi.OP_APPLY_T, lv.A.T @ x)):
            got = c.lv_vec(l, sa.level_apply(c.G, l, op, xb, (mz, my, mx), precision))
            assert emax(got, want) <= tol, (name, l, op, emax(got, want))
        if l == nl - 1:
            continue
        got = c.lv_vec(l, sa.level_apply(c.G, l, sa.capi.OP_PRESMOOTH, xb, (mz, my, mx), precision))
        want = amg.chebyshev(lv, x, None, c.H.opts.cheb_degree, c.H.opts.cheb_ratio)
        assert emax(got, want) <= tol_smooth, (name, l, "presmooth", emax(got, want))
        nx_, ny_, nz_ = c.H.levels[l + 1].dims
        got = c.lv_vec(l + 1, sa.level_apply(c.G, l, sa.capi.OP_RESTRICT, xb, (nz_, ny_, nx_), precision))
        assert emax(got, lv.P.T @ x) <= tol, (name, l, "restrict", emax(got, lv.P.T @ x))
        v = rng.uniform(-1, 1, c.H.levels[l + 1].n)
        got = c.lv_vec(l, sa.level_apply(c.G, l, sa.capi.OP_PROLONG, c.lv_box(l + 1, v), (mz, my, mx), precision))
        assert emax(got, lv.P @ v) <= tol, (name, l, "prolong", emax(got, lv.P @ v))


@pytest.mark.parametrize("name,wide", LANES)
@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_vcycle(name, wide, precision):
    c = case(name, precision, wide=wide)
    r = W.random_box_vector(c.dims, 5) * c.sys.dom.mask
    want = amg.vcycle(c.H, c.sys.gather(r))
    z = torch.zeros(np.prod(c.dims), dtype=torch.float64, device=_dev())
    sa.precond_apply(c.G, c.to_dev(r), z)
    got = c.sys.gather(z.cpu().numpy())
    tol = 1e-11 if precision == W.PREC_FP64 else 1e-4
    print(f"[{name}] vcycle emax={emax(got, want):.2e}", flush=True)
    assert emax(got, want) <= tol


def test_operator_apply_device():
    c = case("ell70_quad")
    x = W.random_box_vector(c.dims, 9) * c.sys.dom.mask
    y = torch.zeros(np.prod(c.dims), dtype=torch.float64, device=_dev())
    sa.operator_apply(c.G, c.to_dev(x), y)
    got = y.cpu().numpy().reshape(c.dims[::-1])
    assert rel(c.sys.gather(got), c.sys.As @ c.sys.gather(x)) <= 1e-14
    assert np.all(got[~c.sys.dom.mask] == 0)


# ------------------------------------------------------------------ full solves


def gpu_solve(c, b, x0=None, tol=1e-8, max_iter=500):
    x = torch.zeros(np.prod(c.dims), dtype=torch.float64, device=_dev())
    res = sa.solve(c.G, c.to_dev(b), x, None if x0 is None else c.to_dev(x0), tol, max_iter)
    return x.cpu().numpy().reshape(c.dims[::-1]), res


@pytest.mark.parametrize("name,wide", LANES)
def test_solve_fp64_matches_oracle(name, wide):
    c = case(name, wide=wide)
    o = solve.solve(c.sys, c.H, c.b, tol=1e-8)
    xo = c.sys.scatter(operator.unscale(c.sys, o.x))
    xg, res = gpu_solve(c, c.b)
    print(f"[{name}] oracle it={o.iterations} gpu it={res['iterations']} rel_true={res['rel_res_true']:.2e}")
    assert res["status"] == 0 and o.status == pcg.OK
    assert abs(res["iterations"] - o.iterations) <= 1
    assert rel(c.sys.gather(xg), c.sys.gather(xo)) <= 1e-8
    assert res["rel_res_true"] <= 1e-8
    assert np.all(xg[~c.sys.dom.mask] == 0)


@pytest.mark.parametrize("name,wide", LANES)
def test_solve_mixed_matches_tight_oracle(name, wide):
    c = case(name, W.PREC_MIXED, wide=wide)
    ref = solve.solve(c.sys, c.H, c.b, tol=1e-13)
    xref = operator.unscale(c.sys, ref.x)
    o8 = operator.unscale(c.sys, solve.solve(c.sys, c.H, c.b, tol=1e-8).x)
    xg, res = gpu_solve(c, c.b)
    err = rel(c.sys.gather(xg), xref)
    print(f"[{name}] mixed it={res['iterations']} err={err:.2e} oracle-1e-8 err={rel(o8, xref):.2e}")
    assert res["status"] == 0 and res["rel_res_true"] <= 1e-8
    assert err <= 1e-6


@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_solve_start_paths_agree(precision):
    """A start without an initial guess takes one fused pass on 16-byte lanes when b is
    16-byte aligned, else the two-pass start (b~ and x, then r = b~ with its partials):
    both give bitwise the same solve."""
    c = case("ell68_quad", precision, wide=2)
    n = int(np.prod(c.dims))
    b = c.to_dev(c.b)
    buf = torch.zeros(n + 1, dtype=torch.float64, device=_dev())
    buf[1:] = b
    b_odd = buf[1:]  # 8 bytes past a 16-byte boundary
    assert b.data_ptr() % 16 == 0 and b_odd.data_ptr() % 16 == 8
    x1 = torch.zeros(n, dtype=torch.float64, device=_dev())
    x2 = torch.zeros(n, dtype=torch.float64, device=_dev())
    r1 = sa.solve(c.G, b, x1, tol=1e-8)
    r2 = sa.solve(c.G, b_odd, x2, tol=1e-8)
    assert r1["status"] == 0 and r2["status"] == 0
    assert r1["iterations"] == r2["iterations"]
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_ring_length_leaves_the_iterates_unchanged(precision):
    """The ring of CG directions on 16-byte lanes (2, 5, 16 or the automatic 32): x takes
    the same updates in the same order however often it is flushed, so every length gives
    bitwise the same solve."""
    base = None
    for ring in (0, 2, 5, 16):
        c = case("ell68_quad", precision, wide=2, ring=ring)
        xg, res = gpu_solve(c, c.b)
        print(f"[ring {ring} prec={precision}] it={res['iterations']}", flush=True)
        assert res["status"] == 0
        if base is None:
            base = (xg, res["iterations"])
        else:
            assert res["iterations"] == base[1] and np.array_equal(xg, base[0]), ring


@pytest.mark.parametrize("precision", [W.PREC_MIXED, W.PREC_FP64])
@pytest.mark.parametrize("wide", [0, 2])
def test_solve_stopped_early(wide, precision):
    """A solve stopped by max_iter (NOT_CONVERGED) after k steps, on both CG forms: the
    fused one (one node per lane, x updated by the next step) and the ring of directions
    (16-byte lanes, x updated from the ring when it is full and before x is read).  The
    returned x carries every step: the reported true residual, which the oracle recomputes
    from x, agrees with the recursive one (a missing alpha p would leave a residual of an
    earlier step's size), and a restart from x converges to the oracle's solution."""
    c = case("ell68_quad", precision, wide=wide, ring=16 if wide else 0)
    xref = operator.unscale(c.sys, solve.solve(c.sys, c.H, c.b, tol=1e-13).x)
    # k = 20 > 16 directions (a ring of 16 on the 16-byte lanes): the ring is flushed once
    # mid-solve (at a tolerance the solve
    # cannot reach, so it still stops by max_iter); its residual is deep, so the two
    # residuals and the oracle's are compared more loosely there
    for k, tol in ((1, 1e-8), (2, 1e-8), (5, 1e-8), (20, 1e-15)):
        xk, rk = gpu_solve(c, c.b, tol=tol, max_iter=k)
        r, bn = operator.scaled_residual(c.sys.dom, c.variant, xk, c.b)
        rel_o = np.linalg.norm(r) / bn
        print(f"[stop {k} wide={wide} prec={precision}] true={rk['rel_res_true']:.6e} recursive="
              f"{rk['rel_res_recursive']:.6e} oracle={rel_o:.6e}", flush=True)
        assert rk["status"] == sa.capi.NOT_CONVERGED and rk["iterations"] == k
        loose = k > 10
        assert abs(rk["rel_res_true"] - rk["rel_res_recursive"]) <= (1e-3 if loose else 1e-6) * rk["rel_res_true"]
        assert abs(rel_o - rk["rel_res_true"]) <= (1e-4 if loose else 1e-7) * rel_o
        assert np.all(xk[~c.sys.dom.mask] == 0)
        x2, r2 = gpu_solve(c, c.b, x0=xk)
        assert r2["status"] == 0 and r2["rel_res_true"] <= 1e-8
        assert rel(c.sys.gather(x2), xref) <= 1e-6


def test_solve_edge_cases():
    c = case("cyl33_lin")
    xz, r0 = gpu_solve(c, np.zeros(c.dims[::-1]))
    assert r0["iterations"] == 0 and r0["status"] == 0 and np.all(xz == 0)
    x, full = gpu_solve(c, c.b)
    _, warm = gpu_solve(c, c.b, x0=x)
    assert warm["iterations"] == 0
    _, near = gpu_solve(c, c.b, x0=x * (1 + 1e-5))
    assert 0 < near["iterations"] < full["iterations"]
    _, one = gpu_solve(c, c.b, max_iter=1)
    assert one["status"] == sa.capi.NOT_CONVERGED and one["iterations"] == 1
    bad = c.b.copy()
    k, j, i = [v[0] for v in np.nonzero(c.sys.dom.mask)]
    bad[k, j, i] = np.nan
    _, nanres = gpu_solve(c, bad)
    assert nanres["status"] == sa.capi.NONFINITE
    # NaN at a node that is not an unknown is ignored
    bad2 = c.b.copy()
    bad2[0, 0, 0] = np.nan
    x2, r2 = gpu_solve(c, bad2)
    assert r2["status"] == 0 and np.array_equal(x2, x)


def test_single_level_and_other_degrees():
    shape = W.Shape.cylinder(1.0, 2.0)
    for (n, nz, deg, mc) in ((11, 9, 2, 1000), (25, 21, 1, 200), (25, 21, 3, 200)):
        opts = amg.Options(max_coarse=mc, cheb_degree=deg)
        s_, H = solve.build(shape, n, n, nz, W.VARIANT_QUAD, opts)
        G = sa.setup(sa.domain_for(shape, n, n, nz), W.VARIANT_QUAD,
                     sa.default_options(max_coarse=mc, cheb_degree=deg))
        b = W.rhs(W.small(shape, n, n, nz, W.VARIANT_QUAD))
        o = solve.solve(s_, H, b)
        x = torch.zeros(n * n * nz, dtype=torch.float64, device=_dev())
        res = sa.solve(G, torch.from_numpy(b.reshape(-1)).to(_dev()), x)
        xo = operator.unscale(s_, o.x)
        assert res["status"] == 0 and abs(res["iterations"] - o.iterations) <= 1
        assert rel(s_.gather(x.cpu().numpy()), xo) <= 1e-8, (n, deg)
        assert sa.hierarchy_info(G)["n_levels"] == len(H.levels)


def _check_coarse_inverse(G, lv):
    """The direct coarse solver's explicit inverse against the inverse of the oracle's
    coarsest operator, element by element, and A_c G = I."""
    rows, inv = sa.coarse_inverse(G)
    assert np.array_equal(rows, lv.lin)
    Ac = lv.A.toarray()
    want = np.linalg.inv(Ac)
    # both inverses carry rounding of about cond(A_c) n eps relative to max |A_c^-1|
    assert emax(inv, want) <= 1e-12, (lv.n, emax(inv, want))
    assert np.abs(Ac @ inv - np.eye(lv.n)).max() <= 1e-12 * np.abs(Ac).sum(axis=1).max()


@pytest.mark.parametrize("name", list(CASES))
def test_coarse_inverse_matches_oracle(name):
    """Blocked Gauss-Jordan on the matrix cores: coarsest levels of 64..996 unknowns (2 to
    32 blocks of 32 pivots, ragged last blocks)."""
    c = case(name)
    _check_coarse_inverse(c.G, c.H.levels[-1])


def test_coarse_inverse_single_level_and_small():
    """Single-level hierarchies (483 and 2,509 unknowns, the inverse of the level-0
    operator) and a coarsest level of 27 unknowns (one partial block)."""
    shape = W.Shape.cylinder(1.0, 2.0)
    for (n, nz, mc, size) in ((11, 9, 1000, 483), (17, 15, 8000, 2509), (25, 21, 200, 27)):
        print(f"[case] cylinder {n}x{n}x{nz} max_coarse={mc}", flush=True)
        _, H = solve.build(shape, n, n, nz, W.VARIANT_QUAD, amg.Options(max_coarse=mc))
        G = sa.setup(sa.domain_for(shape, n, n, nz), W.VARIANT_QUAD,
                     sa.default_options(max_coarse=mc))
        assert H.levels[-1].n == size
        _check_coarse_inverse(G, H.levels[-1])
        sa.destroy(G)


def test_coarse_inverse_absent_for_gauss_seidel():
    c = case("cyl33_lin", gs=True)
    with pytest.raises(sa.SaamgError):
        sa.coarse_inverse(c.G)


def test_batched_states_equal_alone():
    """Each request's result is bitwise the same alone and inside a batch."""
    cs = [case("cyl33_lin", W.PREC_MIXED), case("ell70_quad", W.PREC_MIXED),
          case("boxbore_lin", W.PREC_MIXED)]
    alone = []
    for c in cs:
        x, _ = gpu_solve(c, c.b)
        alone.append(x)
    streams = [torch.cuda.Stream() for _ in cs]
    states = [sa.state_create(c.G, c.to_dev(c.b), stream=s.cuda_stream) for c, s in zip(cs, streams)]
    for _ in range(200):
        if sa.batch_step(states) == len(states):
            break
    for c, st, xa in zip(cs, states, alone):
        done, res = sa.state_query(st)
        assert done and res["status"] == 0
        x = torch.zeros(np.prod(c.dims), dtype=torch.float64, device=_dev())
        torch.cuda.synchronize()  # the fill runs on torch's stream, the finish on the state's
        sa.state_finish(st, x)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy().reshape(c.dims[::-1]), xa)
        sa.state_destroy(st)


# ------------------------------------------------------------------ Gauss-Seidel coarse solver


@pytest.mark.parametrize("name", ["ell70_quad", "cyl_robin_lin"])
def test_gauss_seidel_coarse_solver(name):
    """The iterative coarse level solver (three coloured Gauss-Seidel sweeps): one V-cycle
    and the full fp64 solve against the oracle with the same option."""
    c = case(name, gs=True)
    assert c.info["n_levels"] > 1
    r = W.random_box_vector(c.dims, 6) * c.sys.dom.mask
    want = amg.vcycle(c.H, c.sys.gather(r))
    z = torch.zeros(np.prod(c.dims), dtype=torch.float64, device=_dev())
    sa.precond_apply(c.G, c.to_dev(r), z)
    assert rel(c.sys.gather(z.cpu().numpy()), want) <= 1e-11
    o = solve.solve(c.sys, c.H, c.b, tol=1e-8)
    xo = operator.unscale(c.sys, o.x)
    xg, res = gpu_solve(c, c.b)
    print(f"[{name} gs] oracle it={o.iterations} gpu it={res['iterations']}")
    assert res["status"] == 0 and abs(res["iterations"] - o.iterations) <= 1
    assert rel(c.sys.gather(xg), xo) <= 1e-8
    cm = case(name, W.PREC_MIXED, gs=True)
    xm, resm = gpu_solve(cm, cm.b)
    assert resm["status"] == 0 and rel(cm.sys.gather(xm), xo) <= 1e-6
