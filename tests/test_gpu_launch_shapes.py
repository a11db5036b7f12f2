"""GPU parity in the level-0 launch shapes of the full-size problems, element by element.

The level-0 solve kernels run on one of two lane layouts.  With one node per lane they
tile the box into blocks of `l0_tile_x` 64-node segments of a line and `l0_planes`
z-planes.  On 16-byte lanes (`l0_wide` = 2, the automatic choice for the 256x256x768
ellipse and the 192x192x1024 cylinder) a wavefront spans 256 (fp32) or 128 (fp64) nodes
of a line, and a block 8 (fp32) or 16 (fp64) planes there; lines longer than a span
take several wavefronts that exchange their edge nodes.  The small parity cases reach
none of this.  This file takes an ellipse lattice the oracle solves in seconds but with
lines of 264 = 4*64 + 8 nodes (one-node lanes: a ragged fifth segment; 16-byte lanes: a
second fp32 span of 2 lanes and a third fp64 span of 4) and 70 planes (ragged slabs for
every planes-per-block), and checks every level-0 step and the solves against the oracle
in each launch shape, including the extremes 2 and 32 planes (capped at 14 / 30 planes
on 16-byte lanes).

Tolerances (max |got - want| over max |want|): fp64 1e-12 (components; summation order
only) and 1e-11 (V-cycle); fp32 components 2e-5 (unit roundoff 6e-8 times a few dozen
terms of bounded size per output) and 1e-4 for the V-cycle (rounding carried through
every level and the coarse solve); solves 1e-8 (fp64, iterations +-1) and 1e-6 (mixed
against the oracle's 1e-13 solution).
"""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import amg, operator, pcg, solve

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")

pytestmark = pytest.mark.gpu

SHAPE = W.Shape.ellipse(1.0, 0.3, 1.4)
DIMS = (264, 32, 70)
# (lanes, planes per block, segments per block): one-node lanes in five tilings, then
# 16-byte lanes with 2, 8, 16 and 32 planes asked for
SHAPES = [(1, 2, 4), (1, 16, 4), (1, 32, 4), (1, 16, 2), (1, 16, 1),
          (2, 2, 0), (2, 8, 0), (2, 16, 0), (2, 32, 0)]


def _dev():
    return torch.device("cuda:0")


@functools.lru_cache(maxsize=1)
def oracle():
    sys_, H = solve.build(SHAPE, *DIMS, W.VARIANT_QUAD)
    b = W.rhs(W.small(SHAPE, *DIMS, W.VARIANT_QUAD))
    o = solve.solve(sys_, H, b, tol=1e-8)
    tight = solve.solve(sys_, H, b, tol=1e-13)
    return sys_, H, b, o, tight


def emax(got, want):
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


def _setup(wide, planes, tile, precision):
    o = sa.default_options(precision=precision, l0_planes=planes, l0_tile_x=tile, l0_wide=wide)
    G = sa.setup(sa.domain_for(SHAPE, *DIMS), W.VARIANT_QUAD, o)
    info = sa.hierarchy_info(G)
    assert info["l0_planes"] == planes and info["l0_wide"] == int(wide == 2)
    if wide == 1:
        assert info["l0_tile_x"] == tile
    else:
        assert info["l0_wide_planes"] == [min(planes, 14), min(planes, 30)]
    return G


def test_automatic_shape_of_the_full_size_problems():
    """The shapes this file forces are the ones the full-size problems get by themselves."""
    for name, want in (("ell256_mixed", (16, 4)), ("cyl192_mixed", (16, 2))):
        w = W.by_name(name)
        G = sa.setup(sa.domain_for(w.shape, w.nx, w.ny, w.nz), w.variant,
                     sa.default_options(precision=sa.MIXED))
        info = sa.hierarchy_info(G)
        print(name, info["l0_planes"], info["l0_tile_x"], info["l0_wide"],
              info["l0_wide_planes"], flush=True)
        assert (info["l0_planes"], info["l0_tile_x"]) == want, name
        assert info["l0_wide"] == 1 and info["l0_wide_planes"] == [8, 16], name
        # the cross-section repeats along the pipe: the level-0 table holds the rows of a
        # few planes (lines equal to the line below share its rows)
        print(name, "table rows", info["table_rows"][0], "irregular rows", info["n_irregular"],
              flush=True)
        assert 0 < info["table_rows"][0] < info["n_irregular"] // 4, name
        sa.destroy(G)


@pytest.mark.parametrize("wide,planes,tile", SHAPES)
@pytest.mark.parametrize("precision", [sa.FP64, sa.MIXED])
def test_level0_steps_elementwise(wide, planes, tile, precision):
    print(f"[case] launch shape lanes={wide} planes={planes} tile_x={tile} precision={precision}",
          flush=True)
    sys_, H, _, _, _ = oracle()
    G = _setup(wide, planes, tile, precision)
    lv, lc = H.levels[0], H.levels[1]
    mx, my, mz = lv.dims
    cx, cy, cz = lc.dims
    rng = np.random.default_rng(41)
    x = rng.uniform(-1, 1, lv.n)
    xb = sys_.scatter(x)
    v = rng.uniform(-1, 1, lc.n)
    vb = np.zeros(cx * cy * cz)
    vb[lc.lin] = v
    vb = vb.reshape(cz, cy, cx)
    fp64 = precision == sa.FP64
    tol = 1e-12 if fp64 else 2e-5
    gat = lambda a: a.reshape(-1)[lv.lin]
    checks = {
        "A": (gat(sa.level_apply(G, 0, sa.capi.OP_APPLY, xb, (mz, my, mx), precision)), lv.A @ x),
        "AT": (gat(sa.level_apply(G, 0, sa.capi.OP_APPLY_T, xb, (mz, my, mx), precision)), lv.A.T @ x),
        "presmooth": (gat(sa.level_apply(G, 0, sa.capi.OP_PRESMOOTH, xb, (mz, my, mx), precision)),
                      amg.chebyshev(lv, x, None, H.opts.cheb_degree, H.opts.cheb_ratio)),
        "restrict": (sa.level_apply(G, 0, sa.capi.OP_RESTRICT, xb, (cz, cy, cx), precision).reshape(-1)[lc.lin],
                     lv.P.T @ x),
        "prolong": (gat(sa.level_apply(G, 0, sa.capi.OP_PROLONG, vb, (mz, my, mx), precision)), lv.P @ v),
    }
    worst = {k: emax(g, w) for k, (g, w) in checks.items()}
    r = W.random_box_vector(DIMS, 43) * sys_.dom.mask
    z = torch.zeros(int(np.prod(DIMS)), dtype=torch.float64, device=_dev())
    sa.precond_apply(G, torch.from_numpy(r.reshape(-1)).to(_dev()), z)
    worst["vcycle"] = emax(sys_.gather(z.cpu().numpy()), amg.vcycle(H, sys_.gather(r)))
    print({k: f"{e:.2e}" for k, e in worst.items()}, flush=True)
    for k, e in worst.items():
        lim = (1e-11 if fp64 else 1e-4) if k == "vcycle" else (1e-4 if (k == "presmooth" and not fp64) else tol)
        assert e <= lim, (k, e)
    sa.destroy(G)


@pytest.mark.parametrize("wide,planes,tile", SHAPES)
def test_solves_against_oracle(wide, planes, tile):
    print(f"[case] solves lanes={wide} planes={planes} tile_x={tile}", flush=True)
    sys_, H, b, o, tight = oracle()
    xo = operator.unscale(sys_, o.x)
    xt = operator.unscale(sys_, tight.x)
    bt = torch.from_numpy(b.reshape(-1)).to(_dev())
    for precision in (sa.FP64, sa.MIXED):
        G = _setup(wide, planes, tile, precision)
        x = torch.zeros(int(np.prod(DIMS)), dtype=torch.float64, device=_dev())
        res = sa.solve(G, bt, x, tol=1e-8)
        xg = x.cpu().numpy()
        assert res["status"] == 0 and res["rel_res_true"] <= 1e-8
        assert np.all(xg.reshape(DIMS[::-1])[~sys_.dom.mask] == 0)
        if precision == sa.FP64:
            err = np.linalg.norm(sys_.gather(xg) - xo) / np.linalg.norm(xo)
            print(f"fp64 oracle it={o.iterations} gpu it={res['iterations']} err={err:.2e}", flush=True)
            assert o.status == pcg.OK and abs(res["iterations"] - o.iterations) <= 1 and err <= 1e-8
        else:
            err = np.linalg.norm(sys_.gather(xg) - xt) / np.linalg.norm(xt)
            print(f"mixed it={res['iterations']} err={err:.2e}", flush=True)
            assert err <= 1e-6
        sa.destroy(G)
