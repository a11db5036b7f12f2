"""Continuous-batching server on the GPU: every result equals the same solve run alone,
and the HBM budget caps how many solves share the device."""
import dataclasses

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")
from paper_0907_4863_amd import serve  # noqa: E402

pytestmark = pytest.mark.gpu


def _stream(n=8, seed=21):
    """C4's mix (edges 32..160) plus the largest cross-section of the range and two more
    requests of the first geometry with other bunches (hierarchy cache and warm starts)."""
    reqs = W.serving_stream(n_requests=n, qps=200.0, seed=seed, edge_lo=32, edge_hi=160)
    t = reqs[-1].arrival_s
    big = W.Workload("edge160", W.serving_shape(W.ELLIPSE, 2), 160, 160, 320, W.VARIANT_LIN,
                     W.PREC_MIXED, bunch=W.Bunch(100_000, (0.1, 0.06, 0.3), seed=999))
    reqs.append(W.Request(n, t + 0.001, big))
    w0 = reqs[0].workload
    for k in (1, 2):
        again = dataclasses.replace(w0, name=f"{w0.name}_again{k}",
                                    bunch=dataclasses.replace(w0.bunch, seed=2000 + k))
        reqs.append(W.Request(n + k, t + 0.002 * k, again))
    return reqs


def _alone(w, b, x0=None):
    dev = torch.device("cuda:0")
    H = sa.setup(sa.domain_for(w.shape, w.nx, w.ny, w.nz), w.variant,
                 sa.default_options(precision=w.precision))
    x = torch.zeros(w.box_nodes, dtype=torch.float64, device=dev)
    x0d = None if x0 is None else torch.from_numpy(np.ascontiguousarray(x0)).to(dev)
    res = sa.solve(H, torch.from_numpy(b.reshape(-1)).to(dev), x, x0d, tol=1e-8)
    sa.destroy(H)
    return x.cpu().numpy(), res


def test_served_results_equal_alone():
    """Each served result is bitwise the same request solved alone from the same initial
    guess (zero, or the resident solution it was started from)."""
    reqs = _stream()
    rhs = {r.rid: W.rhs(r.workload) for r in reqs}
    eng = serve.GpuEngine(keep_solutions=True)
    # three hierarchies built at once on worker threads beside the stepping
    srv = serve.Server(serve.ServeConfig(max_active=6, precision=sa.MIXED, setup_workers=3), eng)
    recs = {r.rid: r for r in srv.run(reqs, rhs_of=lambda q: rhs[q.rid])}
    srv.close()
    print(serve.summarize(list(recs.values())), "max concurrent", srv.max_concurrent, flush=True)
    assert srv.max_concurrent >= 2
    assert any(r.cache_hit for r in recs.values())
    assert any(r.warm_from >= 0 for r in recs.values())
    for q in reqs:
        r = recs[q.rid]
        assert r.status == 0 and r.rel_res <= 1e-8
        x0 = None if r.warm_from < 0 else recs[r.warm_from].x
        x, res = _alone(q.workload, rhs[q.rid], x0)
        print(f"rid={q.rid} {q.workload.nx}x{q.workload.ny}x{q.workload.nz} it={r.iterations} "
              f"warm_from={r.warm_from}", flush=True)
        assert res["iterations"] == r.iterations
        assert np.array_equal(x, r.x), q.rid


def test_budget_caps_concurrency():
    reqs = _stream(6, seed=5)
    rhs = {r.rid: W.rhs(r.workload) for r in reqs}
    big = max(sum(sa.footprint_bytes(q.workload.nx, q.workload.ny, q.workload.nz,
                                     q.workload.variant, sa.MIXED)) for q in reqs)
    eng = serve.GpuEngine()
    srv = serve.Server(serve.ServeConfig(hbm_budget_bytes=2 * big + 1, max_active=8,
                                         precision=sa.MIXED), eng)
    recs = srv.run(reqs, rhs_of=lambda q: rhs[q.rid])
    srv.close()
    assert all(r.status == 0 for r in recs) and len(recs) == len(reqs)
    assert srv.peak_used <= 2 * big + 1
