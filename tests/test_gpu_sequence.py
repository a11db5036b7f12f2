"""GPU: sequences of related solves (Section 5.2) against the oracle.

An elongating pipe: the 33^3 cylinder lattice with the length growing by 4% per step, so
h_z changes while the unknowns and near-wall rows stay; the bunch stretches with it.

* saamg_set_operator (reuse of the preconditioner): the operator the CG iteration uses is
  the new geometry's (scaled operator and scaling element by element against the
  oracle's, 1e-14), the preconditioner is bitwise the old one, and the solve reaches the
  oracle's 1e-13 solution of the new geometry to 1e-6 (the mixed-precision bar: PCG with
  another preconditioner stops at the same relative residual, not the same iterate);
  saamg_refresh then gives bitwise the fresh hierarchy's solve.
* SolveSequence: in every mode each step's solution matches the oracle's (1e-6); reusing
  the preconditioner with an iteration limit just below the largest count of an untriggered
  run rebuilds after every solve above the limit, and only then.
"""
import numpy as np
import pytest

import workloads as W
from oracle import operator, solve

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")
from paper_0907_4863_amd import sequence  # noqa: E402

pytestmark = pytest.mark.gpu

N = 33
LENGTHS = [2.0 * (1 + 0.04 * k) for k in range(8)]


def _dev():
    return torch.device("cuda:0")


def _case(k):
    shape = W.Shape.cylinder(1.0, LENGTHS[k])
    return shape, W.rhs(W.small(shape, N, N, N, W.VARIANT_LIN))


def _oracle(k):
    shape, b = _case(k)
    sys_, H = solve.build(shape, N, N, N, W.VARIANT_LIN)
    x = operator.unscale(sys_, solve.solve(sys_, H, b, tol=1e-13).x)
    return sys_, x


def _to(v):
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64).reshape(-1)).to(_dev())


def test_set_operator_keeps_the_preconditioner_and_takes_the_new_operator():
    print("[case] set_operator on the 33^3 cylinder, length 2 -> 2.24", flush=True)
    s0, b0 = _case(0)
    s6, b6 = _case(6)
    d0 = sa.domain_for(s0, N, N, N)
    d6 = sa.domain_for(s6, N, N, N)
    G = sa.setup(d0, W.VARIANT_LIN, sa.default_options())
    F0 = sa.setup(d0, W.VARIANT_LIN, sa.default_options())
    sa.set_operator(G, d6)
    sys6, x6 = _oracle(6)
    x = W.random_box_vector((N, N, N), 3) * sys6.dom.mask
    y = torch.zeros(N ** 3, dtype=torch.float64, device=_dev())
    sa.operator_apply(G, _to(x), y)
    want = sys6.As @ sys6.gather(x)
    assert np.abs(sys6.gather(y.cpu().numpy()) - want).max() <= 1e-14 * np.abs(want).max()
    sig = torch.zeros_like(y)
    sa.scaling(G, sig)
    assert np.abs(sig.cpu().numpy() - sys6.scatter(sys6.sigma).reshape(-1)).max() <= 1e-15 * sys6.sigma.max()
    r = _to(W.random_box_vector((N, N, N), 4) * sys6.dom.mask)
    za, zb = torch.zeros_like(y), torch.zeros_like(y)
    sa.precond_apply(G, r, za)
    sa.precond_apply(F0, r, zb)
    assert torch.equal(za, zb)  # the preconditioner is the one built for length 2
    xs = torch.zeros_like(y)
    res = sa.solve(G, _to(b6), xs, tol=1e-8)
    err = np.linalg.norm(sys6.gather(xs.cpu().numpy()) - x6) / np.linalg.norm(x6)
    F6 = sa.setup(d6, W.VARIANT_LIN, sa.default_options())
    xf = torch.zeros_like(y)
    rf = sa.solve(F6, _to(b6), xf, tol=1e-8)
    print(f"reused preconditioner: {res['iterations']} it, err {err:.1e}; fresh: "
          f"{rf['iterations']} it", flush=True)
    assert res["status"] == 0 and res["rel_res_true"] <= 1e-8 and err <= 1e-6
    sa.refresh(G, d6)
    xr = torch.zeros_like(y)
    rr = sa.solve(G, _to(b6), xr, tol=1e-8)
    assert rr["iterations"] == rf["iterations"] and torch.equal(xr, xf)
    for H in (G, F0, F6):
        sa.destroy(H)


def _run(mode, max_iterations=None, growth=None, check=True):
    seq = sequence.SolveSequence(W.VARIANT_LIN, sa.default_options(), mode=mode,
                                 max_iterations=max_iterations, growth=growth)
    for k in range(len(LENGTHS)):
        shape, b = _case(k)
        rec = seq.step(sa.domain_for(shape, N, N, N), _to(b))
        if check:
            sys_, xo = _oracle(k)
            err = np.linalg.norm(sys_.gather(seq.x.cpu().numpy()) - xo) / np.linalg.norm(xo)
            print(f"step {k}: it={rec.iterations} rebuilt={rec.rebuilt} trigger={rec.trigger} "
                  f"err={err:.1e}", flush=True)
            assert rec.status == 0 and rec.rel_res <= 1e-8 and err <= 1e-6
    seq.close()
    return seq.records


@pytest.mark.parametrize("mode", sequence.MODES)
def test_sequence_modes_match_the_oracle(mode):
    print(f"[case] sequence mode={mode}", flush=True)
    limit = None
    if mode == "preconditioner":
        plain = _run(mode, check=False)  # no limit: the first preconditioner throughout
        assert not any(r.rebuilt for r in plain[1:])
        limit = max(r.iterations for r in plain[1:]) - 1
    recs = _run(mode, max_iterations=limit)
    assert recs[0].rebuilt
    if mode == "rebuild" or mode == "hierarchy":
        assert all(r.rebuilt for r in recs)
    else:
        assert any(r.trigger for r in recs)
        for a, b in zip(recs, recs[1:]):
            assert b.rebuilt == a.trigger  # a rebuild follows every exceeded limit
            assert a.trigger == (a.iterations > limit)
