"""GPU: the opt-in per-class kernel timers (saamg_timer_*).

The timers bind their HIP events to the timed kernel dispatches, so they must
* count one launch per call of each level-0 launcher: the V-cycle's residual, restriction and
  prolongation once per V-cycle (one per PCG iteration plus the initial one), the direction
  update and the residual update once per iteration, and (fp32 directions on 16-byte lanes)
  the x update from the direction ring once per 32 iterations (the ring's default length
  on this machine) and at the end;
* report positive durations whose sum over all classes lies within the timed solve's wall
  time on the same stream, and covers most of the wall time of the same solve run without
  timers (the kernels take as long either way; the untimed ones are the few per-solve set-up
  and copy-out steps);
* record nothing while off.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
sa = pytest.importorskip("paper_0907_4863_amd")

pytestmark = pytest.mark.gpu


def _problem(nx=96):
    dom = sa.domain_for(W.Shape.ellipse(1.0, 0.6, 4.0), nx, 96, 192)
    H = sa.setup(dom, W.VARIANT_QUAD, sa.default_options(precision=W.PREC_MIXED))
    rng = np.random.default_rng(11)
    b = np.where(dom.mask.reshape(-1) > 0, rng.uniform(0, 1, dom.mask.size), 0.0)
    return H, torch.from_numpy(b).cuda()


def _read_all():
    return {k: sa.capi.timer_read(k) for k in sa.capi.TIMER_KINDS}


@pytest.mark.parametrize("nx", [96, 144])
def test_timers_count_launches_and_cover_the_solve(nx):
    print(f"[case] timers, ellipse {nx}x96x192 quadratic mixed", flush=True)
    H, b = _problem(nx)
    wide = sa.hierarchy_info(H)["l0_wide"] == 1
    assert wide == (nx > 128)
    x = torch.zeros_like(b)
    sa.solve(H, b, x, tol=1e-8)  # warm-up
    untimed = []
    for _ in range(2):
        x.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sa.solve(H, b, x, tol=1e-8)
        e1.record()
        torch.cuda.synchronize()
        untimed.append(e0.elapsed_time(e1))
    sa.capi.timer_reset()
    for k in sa.capi.TIMER_KINDS:
        sa.capi.timer_enable(k, True)
    try:
        x.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        res = sa.solve(H, b, x, tol=1e-8)
        e1.record()
        torch.cuda.synchronize()
    finally:
        for k in sa.capi.TIMER_KINDS:
            sa.capi.timer_enable(k, False)
    wall = e0.elapsed_time(e1)
    t = _read_all()
    sa.capi.timer_reset()
    it = res["iterations"]
    assert res["status"] == 0 and it > 0
    for k in ("l0_resid", "l0_restrict", "l0_prolong"):
        assert t[k][1] == it + 1, (k, t[k])
    for k in ("cg_pq", "cg_xr"):
        assert t[k][1] == it, (k, t[k])
    assert t["l0_cheb"][1] > 0 and t["l0_cheb"][1] % (it + 1) == 0
    # the ring of 32 directions flushes before every 33rd direction and once at the end (a
    # replacement of the residual by the true one flushes once more)
    assert t["cg_x"][1] >= (-(-it // 32) if wide else 0), t["cg_x"]
    assert wide or t["cg_x"][1] == 0
    for k, (ms, n, units) in t.items():
        if k == "cg_x" and not wide:
            continue
        assert n > 0 and ms > 0.0 and units > 0, (k, ms, n, units)
    for k in ("l0_cheb", "l0_resid", "l0_restrict", "l0_prolong", "cg_pq", "cg_xr"):
        assert t[k][0] / t[k][1] > 1e-3, (k, t[k])  # > 1 us per launch at this size
    total = sum(ms for ms, _, _ in t.values())
    assert 0.5 * min(untimed) <= total <= 1.02 * wall + 0.05, (total, wall, untimed)


def test_timers_off_record_nothing():
    print("[case] timers off", flush=True)
    H, b = _problem()
    sa.capi.timer_reset()
    x = torch.zeros_like(b)
    sa.solve(H, b, x, tol=1e-8)
    torch.cuda.synchronize()
    for k, v in _read_all().items():
        assert v == (0.0, 0, 0), (k, v)
