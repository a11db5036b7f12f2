"""GPU parity on the method's edge cases, through the C interface.

* Rows with both neighbours of an axis outside the domain: eq. quad_extrapol1 for the
  quadratic rule and the two-sided row (1/s + 1/t)/h^2 of the linear rule.  No pipe on the
  configurations' lattices has them, so the domain is given directly: one-node-wide lines
  along x, y and z and isolated nodes, with seeded wall fractions (some left at 1).  The
  coefficients of every level against the oracle's, element by element, and fp64 and
  mixed solves against the oracle's.
* A coarsening that stalls on level 1: separate 3^3 clusters each become one isolated
  coarse node, which no aggregation reduces, so level 1 is the coarsest (as in the
  oracle's setup).
* A warm start (Section 4: the previous solution as the initial guess): GPU and oracle
  solve from the same x0.

Tolerances as in test_gpu_parity: fp64 coefficients 1e-12 of the largest (1e-14 on level
0), fp64 solutions 1e-8 with iterations +-1, mixed 1e-6 against the oracle's 1e-13
solution.
"""
import numpy as np
import pytest

import workloads as W
from oracle import amg, grid, operator, pcg, solve

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


def oracle_domain(md: W.MaskDomain) -> grid.Domain:
    nx, ny, nz = md.dims
    frac = np.ones((6, nz, ny, nx))
    frac[md.wall_dir.astype(np.int64), md.wall_node // (nx * ny), (md.wall_node // nx) % ny,
         md.wall_node % nx] = md.wall_s
    return grid.Domain(nx, ny, nz, md.h, md.mask.copy(), frac)


def gpu_domain(md: W.MaskDomain) -> "sa.HostDomain":
    return sa.HostDomain(md.mask.astype(np.uint8), md.h, md.wall_node, md.wall_dir, md.wall_s)


def oracle_coef(lv):
    mx, my, mz = lv.dims
    c = amg.coarse_box_coords(lv)
    A = lv.A.tocoo()
    d = c[A.col] - c[A.row]
    k = (d[:, 0] + 1) + 3 * (d[:, 1] + 1) + 9 * (d[:, 2] + 1)
    out = np.zeros((27, mz, my, mx))
    out[k, c[A.row, 2], c[A.row, 1], c[A.row, 0]] = A.data
    return out


def emax(got, want):
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


def gpu_solve(G, dims, b, x0=None, tol=1e-8):
    n = int(np.prod(dims))
    x = torch.zeros(n, dtype=torch.float64, device=_dev())
    to = lambda v: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64).reshape(-1)).to(_dev())
    res = sa.solve(G, to(b), x, None if x0 is None else to(x0), tol, 500)
    return x.cpu().numpy().reshape(dims[::-1]), res


@pytest.mark.parametrize("variant", [W.VARIANT_CONST, W.VARIANT_LIN, W.VARIANT_QUAD])
def test_both_neighbours_outside_rows(variant):
    md = W.thin_lines_domain()
    print(f"[case] thin lines variant={variant}", flush=True)
    dom = oracle_domain(md)
    sys_ = operator.assemble(dom, variant)
    H = amg.setup(sys_.As, md.dims, sys_.idx)
    # the domain has rows of the both-outside kind on every axis
    ks, js, is_ = np.nonzero(md.mask)
    for axis, (dx, dy, dz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        both = ~md.mask[ks - dz, js - dy, is_ - dx] & ~md.mask[ks + dz, js + dy, is_ + dx]
        assert both.sum() >= 10, axis
    G = sa.setup(gpu_domain(md), variant, sa.default_options())
    info = sa.hierarchy_info(G)
    assert info["n_unknowns"] == H.sizes
    for l, lv in enumerate(H.levels):
        e = emax(sa.level_coefficients(G, l, lv.dims), oracle_coef(lv))
        assert e <= (1e-14 if l == 0 else 1e-12), (l, e)
    b = W.random_box_vector(md.dims, 31)
    o = solve.solve(sys_, H, b, tol=1e-8)
    xo = sys_.scatter(operator.unscale(sys_, o.x))
    xg, res = gpu_solve(G, md.dims, b)
    err = np.linalg.norm(sys_.gather(xg) - sys_.gather(xo)) / np.linalg.norm(sys_.gather(xo))
    print(f"fp64 oracle it={o.iterations} gpu it={res['iterations']} err={err:.2e}", flush=True)
    assert o.status == pcg.OK and res["status"] == 0
    assert abs(res["iterations"] - o.iterations) <= 1 and err <= 1e-8
    ref = sys_.gather(sys_.scatter(operator.unscale(sys_, solve.solve(sys_, H, b, tol=1e-13).x)))
    Gm = sa.setup(gpu_domain(md), variant, sa.default_options(precision=sa.MIXED))
    xm, resm = gpu_solve(Gm, md.dims, b)
    errm = np.linalg.norm(sys_.gather(xm) - ref) / np.linalg.norm(ref)
    print(f"mixed it={resm['iterations']} err={errm:.2e}", flush=True)
    assert resm["status"] == 0 and errm <= 1e-6
    sa.destroy(G)
    sa.destroy(Gm)


def test_coarsening_stall_makes_the_level_coarsest():
    md = W.cluster_domain()
    print("[case] 27 clusters, max_coarse 1", flush=True)
    dom = oracle_domain(md)
    sys_ = operator.assemble(dom, W.VARIANT_LIN)
    H = amg.setup(sys_.As, md.dims, sys_.idx, amg.Options(max_coarse=1))
    assert H.sizes == [729, 27]
    G = sa.setup(gpu_domain(md), W.VARIANT_LIN, sa.default_options(max_coarse=1))
    info = sa.hierarchy_info(G)
    assert info["n_levels"] == 2 and info["n_unknowns"] == [729, 27]
    b = W.random_box_vector(md.dims, 32)
    o = solve.solve(sys_, H, b, tol=1e-8)
    xo = sys_.gather(sys_.scatter(operator.unscale(sys_, o.x)))
    xg, res = gpu_solve(G, md.dims, b)
    assert res["status"] == 0 and abs(res["iterations"] - o.iterations) <= 1
    assert np.linalg.norm(sys_.gather(xg) - xo) <= 1e-8 * np.linalg.norm(xo)
    sa.destroy(G)


@pytest.mark.parametrize("precision", [sa.FP64, sa.MIXED])
def test_warm_start_matches_oracle(precision):
    """Both solvers start from x0 = the oracle's solution for the bunch one step earlier
    (shifted by 0.02 along z), as a time step of Section 4 does."""
    shape = W.Shape.ellipse(1.0, 0.6, 4.0)
    nx, ny, nz = 70, 45, 66
    print(f"[case] warm start ellipse {nx}x{ny}x{nz} precision={precision}", flush=True)
    sys_, H = solve.build(shape, nx, ny, nz, W.VARIANT_QUAD)
    w = W.small(shape, nx, ny, nz, W.VARIANT_QUAD)
    b = W.rhs(w)
    x_star = sys_.scatter(operator.unscale(sys_, solve.solve(sys_, H, b, tol=1e-13).x))
    prev = solve.solve(sys_, H, W.rhs(w, shift_z=-0.02), tol=1e-8)
    x0 = sys_.scatter(operator.unscale(sys_, prev.x))
    cold = solve.solve(sys_, H, b, tol=1e-8)
    o = solve.solve(sys_, H, b, x0, tol=1e-8)
    xo = sys_.gather(sys_.scatter(operator.unscale(sys_, o.x)))
    G = sa.setup(sa.domain_for(shape, nx, ny, nz), W.VARIANT_QUAD,
                 sa.default_options(precision=precision))
    xg, res = gpu_solve(G, (nx, ny, nz), b, x0=x0)
    err = np.linalg.norm(sys_.gather(xg) - xo) / np.linalg.norm(xo)
    print(f"oracle cold it={cold.iterations} warm it={o.iterations} gpu it={res['iterations']} "
          f"err={err:.2e}", flush=True)
    assert o.iterations < cold.iterations
    assert res["status"] == 0
    if precision == sa.FP64:
        assert abs(res["iterations"] - o.iterations) <= 1 and err <= 1e-8
    else:
        xs = sys_.gather(x_star)
        assert np.linalg.norm(sys_.gather(xg) - xs) <= 1e-6 * np.linalg.norm(xs)
    sa.destroy(G)


def test_torch_allocator_option_gives_the_same_solution():
    """saamg_options' allocator callbacks backed by torch's caching allocator: the same
    hierarchy and solution bit for bit as with the library's own pool, and every buffer
    is handed back when the hierarchy is destroyed."""
    shape = W.Shape.ellipse(1.0, 0.6, 4.0)
    nx, ny, nz = 70, 45, 66
    print("[case] torch allocator option", flush=True)
    dom = sa.domain_for(shape, nx, ny, nz)
    b = W.rhs(W.small(shape, nx, ny, nz, W.VARIANT_QUAD))
    al = sa.capi.TorchAllocator()
    xs = []
    for alloc in (None, al):
        G = sa.setup(dom, W.VARIANT_QUAD, sa.default_options(allocator=alloc, precision=sa.MIXED))
        x, res = gpu_solve(G, (nx, ny, nz), b)
        assert res["status"] == 0
        xs.append(x)
        sa.destroy(G)
    torch.cuda.synchronize()
    print(f"torch allocator: {al.n_alloc} allocations, {al.n_free} frees", flush=True)
    assert al.n_alloc > 50 and al.n_free == al.n_alloc and al.outstanding_bytes == 0
    assert np.array_equal(xs[0], xs[1])
