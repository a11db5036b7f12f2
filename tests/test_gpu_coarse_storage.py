"""GPU: the compressed coarse operators (interior stencil + table) apply the same operators as
the full coefficient arrays the Galerkin product writes.

The domain is a hollow pipe: the lattice nodes near the axis are removed, so the node at the
centre of the coarse boxes is not an unknown and the levels have no interior reference row
(every row then comes from the table).  A_l x and A_l^T x from the solve kernels are checked
against sums over the exported full arrays, on every coarse level, in fp64 (1e-12) and with
the fp32 copies (1e-5: single rounding of each coefficient and product, summed over 27
terms).  A solve on the hollow pipe converges in both precisions to the same solution.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")

pytestmark = pytest.mark.gpu


def _hollow_domain(n=41, nz=41, r_in=0.3):
    d = sa.domain_for(W.Shape.cylinder(1.0, 2.0), n, n, nz)
    x = np.linspace(-1.0, 1.0, n)
    inner = (x[None, :] ** 2 + x[:, None] ** 2) < r_in ** 2  # (y, x)
    mask = d.mask.copy()
    mask[:, inner] = 0
    # the constant rule ignores wall fractions, so no wall entries are needed
    e = np.zeros(0)
    return sa.capi.HostDomain(mask, d.h, e.astype(np.int64), e.astype(np.uint8), e)


def _apply_full(coef, x, trans):
    """sum_k A(i, i+o_k) x(i+o_k) (trans: A^T) from [27][mz][my][mx] arrays, zero outside."""
    mz, my, mx = x.shape
    xp = np.zeros((mz + 2, my + 2, mx + 2))
    xp[1:-1, 1:-1, 1:-1] = x
    y = np.zeros_like(x)
    for k in range(27):
        dx, dy, dz = k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1
        xs = xp[1 + dz:1 + dz + mz, 1 + dy:1 + dy + my, 1 + dx:1 + dx + mx]
        if not trans:
            y += coef[k] * xs
        else:  # A^T(i, i+o) = A(i+o, i): the neighbour's coefficient of offset 26-k
            cp = np.zeros((mz + 2, my + 2, mx + 2))
            cp[1:-1, 1:-1, 1:-1] = coef[26 - k]
            y += cp[1 + dz:1 + dz + mz, 1 + dy:1 + dy + my, 1 + dx:1 + dx + mx] * xs
    return y


@pytest.mark.parametrize("precision", [W.PREC_FP64, W.PREC_MIXED])
def test_compressed_coarse_operators_match_full_arrays(precision):
    print(f"[case] hollow pipe 41^3, constant rule, precision {precision}", flush=True)
    dom = _hollow_domain()
    assert dom.mask[20, 20, 20] == 0
    G = sa.setup(dom, W.VARIANT_CONST, sa.default_options(precision=precision, max_coarse=30))
    info = sa.hierarchy_info(G)
    assert info["n_levels"] >= 3
    rng = np.random.default_rng(7)
    tol = 1e-12 if precision == W.PREC_FP64 else 1e-5
    for l in range(1, info["n_levels"]):
        mx, my, mz = info["dims"][l]
        coef = sa.level_coefficients(G, l, (mx, my, mz))
        unk = coef[13] != 0.0
        assert unk.sum() == info["n_unknowns"][l]
        x = np.where(unk, rng.uniform(-1, 1, unk.shape), 0.0)
        for op, trans in ((sa.capi.OP_APPLY, False), (sa.capi.OP_APPLY_T, True)):
            got = sa.level_apply(G, l, op, x, (mz, my, mx), precision)
            want = np.where(unk, _apply_full(coef, x, trans), 0.0)
            assert np.abs(got - want).max() <= tol * np.abs(want).max(), (l, op)


def test_hollow_pipe_solves_in_both_precisions():
    print("[case] hollow pipe solve", flush=True)
    dom = _hollow_domain()
    nbox = dom.mask.size
    rng = np.random.default_rng(8)
    b = torch.from_numpy(np.where(dom.mask.reshape(-1) > 0, rng.uniform(0, 1, nbox), 0.0)).cuda()
    xs = []
    for prec in (W.PREC_FP64, W.PREC_MIXED):
        G = sa.setup(dom, W.VARIANT_CONST, sa.default_options(precision=prec))
        x = torch.zeros_like(b)
        res = sa.solve(G, b, x, tol=1e-10)
        assert res["status"] == 0 and res["rel_res_true"] <= 1e-10
        xs.append(x.cpu().numpy())
    assert np.linalg.norm(xs[1] - xs[0]) <= 1e-8 * np.linalg.norm(xs[0])
