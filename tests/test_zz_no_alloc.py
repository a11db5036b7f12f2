"""GPU: saamg_solve_noalloc, whose work vectors live in the library's static scratch array,
against saamg_solve on the same hierarchies, through the C interface.

Calls in a row on smaller and smaller problems (the array keeps the previous call's
contents, which must not leak into the next), in fp64 and mixed precision; the output
must match saamg_solve's to the parity bar (1e-8 fp64, 1e-6 mixed) with the same
iteration count (the kernels and their order are the same, so it is expected bitwise),
and the call must not go through the allocator.  A warm start is checked the same way,
and a problem too large for the array is refused with SAAMG_INVALID_ARG.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")

pytestmark = pytest.mark.gpu

# larger first, then smaller; the first on 16-byte lanes (nx a multiple of 4 above 128), where
# the allocation-free solve keeps 2 CG directions in its ring against up to 32
CASES = [("ell132_quad", W.Shape.ellipse(1.0, 0.6, 4.0), 132, 45, 40, W.VARIANT_QUAD),
         ("ell70_quad", W.Shape.ellipse(1.0, 0.6, 4.0), 70, 45, 66, W.VARIANT_QUAD),
         ("cyl33_lin", W.Shape.cylinder(1.0, 2.0), 33, 33, 33, W.VARIANT_LIN)]


def _dev():
    return torch.device("cuda:0")


def _rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


@pytest.mark.parametrize("precision", [sa.FP64, sa.MIXED])
def test_noalloc_matches_solve_large_then_small(precision):
    bar = 1e-8 if precision == sa.FP64 else 1e-6
    al = sa.capi.torch_allocator()
    for name, shape, nx, ny, nz, variant in CASES:
        print(f"[case] noalloc {name} precision={precision}", flush=True)
        # the hierarchy's allocator is torch's, whose callbacks count: the call must not use it
        G = sa.setup(sa.domain_for(shape, nx, ny, nz), variant,
                     sa.default_options(allocator="torch", precision=precision))
        b = torch.from_numpy(W.rhs(W.small(shape, nx, ny, nz, variant)).reshape(-1)).to(_dev())
        xa = torch.zeros(nx * ny * nz, dtype=torch.float64, device=_dev())
        ra = sa.solve(G, b, xa, tol=1e-8)
        xn = torch.full_like(xa, float("nan"))  # every entry must be written
        torch.cuda.synchronize()
        n0, f0 = al.n_alloc, al.n_free
        rn = sa.solve_noalloc(G, b, xn, tol=1e-8)
        assert (al.n_alloc, al.n_free) == (n0, f0)
        err = _rel(xn, xa)
        print(f"solve it={ra['iterations']} noalloc it={rn['iterations']} rel={err:.1e} "
              f"bitwise={bool(torch.equal(xn, xa))}", flush=True)
        assert rn["status"] == 0 and rn["iterations"] == ra["iterations"]
        assert rn["rel_res_true"] <= 1e-8 and err <= bar
        # warm start from the solution just computed, perturbed
        x0 = xa * 1.001
        xw = torch.zeros_like(xa)
        rw = sa.solve(G, b, xw, x0=x0, tol=1e-8)
        xwn = torch.zeros_like(xa)
        rwn = sa.solve_noalloc(G, b, xwn, x0=x0, tol=1e-8)
        assert rwn["status"] == 0 and rwn["iterations"] == rw["iterations"]
        assert rw["iterations"] < ra["iterations"] and _rel(xwn, xw) <= bar
        sa.destroy(G)


def test_noalloc_refuses_a_problem_larger_than_its_array():
    w = W.c2_ellipse128()
    print("[case] noalloc refusal on the 128x128x256 ellipse", flush=True)
    G = sa.setup(sa.domain_for(w.shape, w.nx, w.ny, w.nz), w.variant, sa.default_options())
    b = torch.zeros(w.box_nodes, dtype=torch.float64, device=_dev())
    x = torch.zeros_like(b)
    with pytest.raises(sa.SaamgError) as e:
        sa.solve_noalloc(G, b, x)
    assert e.value.status == sa.capi.INVALID_ARG and "scratch" in str(e.value)
    sa.destroy(G)
