"""Continuous-batching server on the GPU: every result equals the same solve run alone,
and the HBM budget caps how many solves share the device."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")
from paper_0907_4863_amd import serve  # noqa: E402

pytestmark = pytest.mark.gpu


def _stream(n=8, seed=21):
    reqs = W.serving_stream(n_requests=n, qps=200.0, seed=seed, edge_lo=20, edge_hi=44)
    # repeat one geometry so the hierarchy cache is exercised
    reqs.append(W.Request(n, reqs[-1].arrival_s + 0.001, reqs[0].workload))
    return reqs


def _alone(w, b):
    dev = torch.device("cuda:0")
    H = sa.setup(sa.domain_for(w.shape, w.nx, w.ny, w.nz), w.variant,
                 sa.default_options(precision=w.precision))
    x = torch.zeros(w.box_nodes, dtype=torch.float64, device=dev)
    res = sa.solve(H, torch.from_numpy(b.reshape(-1)).to(dev), x, tol=1e-8)
    sa.destroy(H)
    return x.cpu().numpy(), res


def test_served_results_equal_alone():
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
    for q in reqs:
        r = recs[q.rid]
        assert r.status == 0 and r.rel_res <= 1e-8
        x, res = _alone(q.workload, rhs[q.rid])
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
