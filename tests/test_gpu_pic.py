"""Particle coupling on the GPU against the oracle: cloud-in-cell deposition (deterministic
fp64) and the field gather E = -grad(phi), on closed and open-ended pipes."""
import numpy as np
import pytest

import workloads as W
from oracle import grid, pic

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")

pytestmark = pytest.mark.gpu

CASES = [
    (W.Shape.cylinder(1.0, 2.0), 41, 41, 61, False),
    (W.Shape.ellipse(1.0, 0.6, 4.0), 48, 30, 70, True),
]


def _dev():
    return torch.device("cuda:0")


def _setup(shape, nx, ny, nz, robin, n=200_000, seed=3):
    dom = sa.domain_for(shape, nx, ny, nz, open_ends=robin)
    origin = (-shape.a, -shape.b, -0.5 * shape.length)
    og = grid.from_shape(shape, nx, ny, nz, robin=robin)
    g = pic.Grid((og.nx, og.ny, og.nz), int(robin), origin, og.h, og.robin_d)
    pts = W.draw_particles(W.Bunch(n, (0.4 * shape.a, 0.4 * shape.b, 0.3 * shape.length), seed))
    return dom, og, g, origin, pts


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("shape,nx,ny,nz,robin", CASES)
def test_deposit_matches_oracle_and_is_deterministic(shape, nx, ny, nz, robin):
    dom, og, g, origin, pts = _setup(shape, nx, ny, nz, robin)
    print(f"[case] deposit {shape.name} {nx}x{ny}x{nz} robin={robin}", flush=True)
    P = sa.pic_create(dom, origin, len(pts))
    pos = torch.from_numpy(pts).to(_dev())
    rho = torch.empty(dom.mask.size, dtype=torch.float64, device=_dev())
    sa.pic_deposit(P, pos, 1.0 / len(pts), rho)
    r1 = rho.cpu().numpy()
    want = pic.deposit(g, pts, 1.0 / len(pts)).reshape(-1)
    assert _rel(r1, want) <= 1e-12
    sa.pic_deposit(P, pos, 1.0 / len(pts), rho)
    assert np.array_equal(rho.cpu().numpy(), r1)
    empty = torch.empty((0, 3), dtype=torch.float64, device=_dev())
    sa.pic_deposit(P, empty, 1.0, rho)
    assert not rho.cpu().numpy().any()


@pytest.mark.parametrize("shape,nx,ny,nz,robin", CASES)
def test_gather_matches_oracle_on_a_solution(shape, nx, ny, nz, robin):
    dom, og, g, origin, pts = _setup(shape, nx, ny, nz, robin, seed=4)
    print(f"[case] gather {shape.name} {nx}x{ny}x{nz} robin={robin}", flush=True)
    P = sa.pic_create(dom, origin, len(pts))
    pos = torch.from_numpy(pts).to(_dev())
    rho = torch.empty(dom.mask.size, dtype=torch.float64, device=_dev())
    sa.pic_deposit(P, pos, 1.0 / len(pts), rho)
    H = sa.setup(dom, W.VARIANT_LIN, sa.default_options())
    phi = torch.zeros_like(rho)
    res = sa.solve(H, rho, phi, tol=1e-10)
    sa.destroy(H)
    assert res["status"] == 0
    E = torch.empty_like(pos)
    sa.pic_gather(P, phi, pos, E)
    want = pic.gather(g, phi.cpu().numpy().reshape(og.mask.shape), og.mask, pts)
    assert _rel(E.cpu().numpy(), want) <= 1e-12
    assert np.abs(want).max() > 0
