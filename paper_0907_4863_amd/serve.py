"""Continuous-batching solve server on one GPU.

Requests (a pipe geometry, a lattice, a right-hand side) arrive over time.  The loop
admits a request as soon as a slot is free and its device footprint fits the HBM budget,
reuses hierarchies cached per geometry (the paper's reuse of the preconditioner across
solves, Section 5, ML variations), keeps the last solution of each cached geometry on the
device and starts the next request of that geometry from it (the warm start of Section 4),
and advances the admitted solves through ``saamg_batch_advance``, which never waits: each
solve owns a stream and steps at its own pace, so a small solve is not held back by a large
one.  Finished solves retire at once and free their memory for queued requests.  Latency
is completion minus arrival.

The device work goes through an engine object (``GpuEngine`` below) so that the
scheduling logic can be exercised without a GPU.  An engine whose ``concurrent_setup`` is
true has the hierarchies of new geometries built on a worker thread, so that the running
solves keep stepping meanwhile; a request waits, with its memory reserved, until its
hierarchy is ready (later requests for the same geometry wait on the same build).
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import threading
import time
from collections import OrderedDict
from typing import Any, Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import capi


@dataclasses.dataclass
class ServeConfig:
    hbm_budget_bytes: int = 64 << 30
    max_active: int = 16
    precision: int = capi.MIXED
    tol: float = 1e-8
    max_iter: int = 500
    cache_hierarchies: bool = True
    # threads building hierarchies (engines with concurrent_setup), each on its own stream
    setup_workers: int = 2
    # keep the last solution of each cached geometry resident and start the next request
    # of that geometry from it (counted in the budget, evicted with the hierarchy)
    warm_start: bool = True
    # host wait between polls when no solve completed a step
    poll_s: float = 50e-6


@dataclasses.dataclass
class Record:
    rid: int
    arrival_s: float
    admit_s: float = float("nan")
    done_s: float = float("nan")
    iterations: int = 0
    status: int = -1
    rel_res: float = float("nan")
    setup_ms: float = 0.0
    cache_hit: bool = False
    warm_from: int = -1       # rid of the solution this request started from (-1: x0 = 0)
    dof: int = 0
    x: Any = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class GpuEngine:
    """Device side of the server: hierarchies, states and steps through the C interface."""

    concurrent_setup = True  # setup() may run on a worker thread beside step()

    def __init__(self, device: int = 0, keep_solutions: bool = False, allocator=None):
        import torch
        self.torch = torch
        self.dev = torch.device(f"cuda:{device}")
        self.keep = keep_solutions
        self.allocator = allocator  # saamg_options allocator (capi.default_options)
        self._streams: List[Any] = []
        self._tls = threading.local()  # one setup stream per worker thread

    def key(self, w) -> Tuple:
        s = w.shape
        return (s.kind, s.a, s.b, s.length, s.bore_r, s.cavity_half_len, w.nx, w.ny, w.nz, w.variant)

    def footprint(self, w, precision: int) -> Tuple[int, int]:
        return capi.footprint_bytes(w.nx, w.ny, w.nz, w.variant, precision)

    def setup(self, w, precision: int):
        dom = capi.domain_for(w.shape, w.nx, w.ny, w.nz)
        st = getattr(self._tls, "stream", None)
        if st is None:
            st = self._tls.stream = self.torch.cuda.Stream(device=self.dev)  # default priority
        H = capi.setup(dom, w.variant,
                       capi.default_options(allocator=self.allocator, precision=precision),
                       stream=st.cuda_stream)
        st.synchronize()  # complete before any state's stream uses H
        info = capi.hierarchy_info(H)
        return H, info["device_bytes"], dom.n_unknowns

    def release_hierarchy(self, H) -> None:
        capi.destroy(H)

    def _stream(self):
        if self._streams:
            return self._streams.pop()
        return self.torch.cuda.Stream(device=self.dev)  # default priority

    def warm_bytes(self, w) -> int:
        """Device bytes of a resident solution of workload w."""
        return 8 * w.nx * w.ny * w.nz

    def start(self, H, b_host: np.ndarray, tol: float, max_iter: int, x0=None):
        """Queue a solve on a stream of its own: the upload of b, the initial residual and
        the first preconditioner are ordered on that stream (no device-wide wait)."""
        torch = self.torch
        st = self._stream()
        with torch.cuda.stream(st):
            b = torch.from_numpy(np.ascontiguousarray(b_host, dtype=np.float64).reshape(-1)).to(self.dev)
        if x0 is not None:
            x0.record_stream(st)  # a resident solution read on this stream
        S = capi.state_create(H, b, x0=x0, tol=tol, max_iter=max_iter, stream=st.cuda_stream)
        return {"S": S, "b": b, "stream": st, "H": H}

    def step(self, handles: Sequence[dict]) -> int:
        """Advance without waiting; returns how many solves completed a step."""
        return capi.batch_advance([h["S"] for h in handles])[1]

    def query(self, h) -> Tuple[bool, dict]:
        return capi.state_query(h["S"])

    def finish(self, h, keep_warm: bool = False):
        """Retire a solve: (host copy of x or None, device x kept for a warm start or None)."""
        torch = self.torch
        x_host = x_dev = None
        if self.keep or keep_warm:
            st = h["stream"]
            with torch.cuda.stream(st):
                x = torch.empty(h["b"].numel(), dtype=torch.float64, device=self.dev)
            capi.state_finish(h["S"], x)  # writes every entry on st and waits for it
            if self.keep:
                x_host = x.cpu().numpy()
            if keep_warm:
                x_dev = x
        capi.state_destroy(h["S"])
        self._streams.append(h["stream"])
        return x_host, x_dev

    def release_warm(self, x) -> None:
        pass  # a torch tensor: its memory returns to the caching allocator when dropped


class Server:
    def __init__(self, cfg: ServeConfig, engine, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.cfg = cfg
        self.eng = engine
        self.clock = clock
        self.sleep = sleep
        # key -> {H, bytes, refs, dof, warm: (device x, rid) or None, warm_bytes}
        self.cache: "OrderedDict[Tuple, dict]" = OrderedDict()
        self.used = 0
        self.peak_used = 0
        self.max_concurrent = 0
        self.rounds = 0
        self.rejected: List[int] = []

    # -------------------------------------------------------------- memory accounting
    def _evict_for(self, need: int) -> None:
        for key in list(self.cache.keys()):
            if self.used + need <= self.cfg.hbm_budget_bytes:
                return
            e = self.cache[key]
            if e["refs"] == 0:
                self._drop(key)

    def _drop(self, key) -> None:
        """Release a cached geometry: its hierarchy and its resident solution."""
        e = self.cache.pop(key)
        self._set_warm(e, None)
        self.eng.release_hierarchy(e["H"])
        self.used -= e["bytes"]

    def _set_warm(self, e: dict, warm) -> None:
        """Replace the resident solution of a cache entry (None: drop it)."""
        if e.get("warm") is not None:
            self.eng.release_warm(e["warm"][0])
            self.used -= e["warm_bytes"]
        e["warm"] = None
        if warm is not None and self.used + e["warm_bytes"] <= self.cfg.hbm_budget_bytes:
            e["warm"] = warm
            self.used += e["warm_bytes"]
            self.peak_used = max(self.peak_used, self.used)
        elif warm is not None:
            self.eng.release_warm(warm[0])

    def _new_entry(self, w, H, hbytes: int, dof: int) -> dict:
        wb = self.eng.warm_bytes(w) if hasattr(self.eng, "warm_bytes") else 0
        return {"H": H, "bytes": hbytes, "refs": 0, "dof": dof, "warm": None, "warm_bytes": wb}

    def _start(self, e: dict, rec: Record, rhs: np.ndarray):
        """Start a request on a cached hierarchy, from its resident solution if any."""
        x0 = None
        if self.cfg.warm_start and e.get("warm") is not None:
            x0, rec.warm_from = e["warm"]
        if x0 is None:
            return self.eng.start(e["H"], rhs, self.cfg.tol, self.cfg.max_iter)
        return self.eng.start(e["H"], rhs, self.cfg.tol, self.cfg.max_iter, x0=x0)

    def _timed_setup(self, w):
        t0 = self.clock()
        r = self.eng.setup(w, self.cfg.precision)
        return r, 1e3 * (self.clock() - t0)

    def _admit_async(self, req, rhs: np.ndarray, now: float, pool, building: dict) -> Optional[dict]:
        """Admission with the hierarchy of a new geometry built on the worker: returns an
        active entry (cached geometry) or a pending one (with the setup's future)."""
        w = req.workload
        key = self.eng.key(w)
        hier_est, state_bytes = self.eng.footprint(w, self.cfg.precision)
        cached = key in self.cache
        new_build = not cached and key not in building
        need = state_bytes + (hier_est if new_build else 0)
        if self.used + need > self.cfg.hbm_budget_bytes:
            self._evict_for(need)
        if self.used + need > self.cfg.hbm_budget_bytes:
            return None
        rec = Record(req.rid, req.arrival_s, admit_s=now)
        self.used += need  # the state, and the hierarchy's estimate until its size is known
        self.peak_used = max(self.peak_used, self.used)
        if cached:
            e = self.cache.pop(key)
            self.cache[key] = e  # most recently used
            rec.cache_hit = True
            e["refs"] += 1
            rec.dof = e["dof"]
            h = self._start(e, rec, rhs)
            return {"rec": rec, "h": h, "key": key, "state_bytes": state_bytes}
        if new_build:
            building[key] = {"fut": pool.submit(self._timed_setup, w), "est": hier_est}
        return {"rec": rec, "key": key, "state_bytes": state_bytes, "rhs": rhs,
                "build": building[key], "builder": new_build, "rec_w": w}

    def _start_pending(self, p: dict, building: dict) -> dict:
        """Start a pending request whose hierarchy is built."""
        key, rec = p["key"], p["rec"]
        if key not in self.cache:  # the first request served by this build
            (H, hbytes, dof), setup_ms = p["build"]["fut"].result()
            self.cache[key] = self._new_entry(p["rec_w"], H, hbytes, dof)
            self.used += hbytes - p["build"]["est"]
            self.peak_used = max(self.peak_used, self.used)
            building.pop(key, None)
        if p["builder"]:
            rec.setup_ms = p["build"]["fut"].result()[1]
        e = self.cache[key]
        e["refs"] += 1
        rec.dof = e["dof"]
        h = self._start(e, rec, p["rhs"])
        return {"rec": rec, "h": h, "key": key, "state_bytes": p["state_bytes"]}

    def _admit(self, req, rhs: np.ndarray, now: float, active: List[dict]) -> Optional[dict]:
        w = req.workload
        key = self.eng.key(w)
        hier_est, state_bytes = self.eng.footprint(w, self.cfg.precision)
        cached = key in self.cache
        need = state_bytes + (0 if cached else hier_est)
        if self.used + need > self.cfg.hbm_budget_bytes:
            self._evict_for(need)
        if self.used + need > self.cfg.hbm_budget_bytes:
            return None
        rec = Record(req.rid, req.arrival_s, admit_s=now)
        if cached:
            e = self.cache.pop(key)
            self.cache[key] = e  # most recently used
            rec.cache_hit = True
        else:
            t0 = self.clock()
            H, hbytes, dof = self.eng.setup(w, self.cfg.precision)
            rec.setup_ms = 1e3 * (self.clock() - t0)
            e = self._new_entry(w, H, hbytes, dof)
            self.cache[key] = e
            self.used += hbytes
        e["refs"] += 1
        rec.dof = e["dof"]
        h = self._start(e, rec, rhs)
        self.used += state_bytes
        self.peak_used = max(self.peak_used, self.used)
        return {"rec": rec, "h": h, "key": key, "state_bytes": state_bytes}

    def _retire(self, a: dict, now: float) -> Record:
        done, res = self.eng.query(a["h"])
        rec = a["rec"]
        rec.done_s = now
        rec.iterations = res["iterations"]
        rec.status = res["status"]
        rec.rel_res = res["rel_res_true"]
        keep_warm = (self.cfg.warm_start and self.cfg.cache_hierarchies and rec.status == capi.OK)
        rec.x, x_dev = self.eng.finish(a["h"], keep_warm)
        self.used -= a["state_bytes"]
        e = self.cache[a["key"]]
        e["refs"] -= 1
        if x_dev is not None:
            self._set_warm(e, (x_dev, rec.rid))
        if not self.cfg.cache_hierarchies and e["refs"] == 0:
            self._drop(a["key"])
        return rec

    # -------------------------------------------------------------- main loop
    def run(self, requests: Sequence, rhs_of: Callable[[Any], np.ndarray]) -> List[Record]:
        """Serve requests (objects with rid, arrival_s, workload) in arrival order."""
        if getattr(self.eng, "concurrent_setup", False):
            with cf.ThreadPoolExecutor(max_workers=self.cfg.setup_workers) as pool:
                return self._run_async(requests, rhs_of, pool)
        queue = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        t0 = self.clock()
        active: List[dict] = []
        out: List[Record] = []
        qi = 0
        while qi < len(queue) or active:
            now = self.clock() - t0
            while qi < len(queue) and queue[qi].arrival_s <= now and len(active) < self.cfg.max_active:
                req = queue[qi]
                a = self._admit(req, rhs_of(req), self.clock() - t0, active)
                if a is None:
                    if not active:
                        # can never fit: reject instead of waiting forever
                        r = Record(req.rid, req.arrival_s, status=capi.NOMEM)
                        r.done_s = self.clock() - t0
                        out.append(r)
                        self.rejected.append(req.rid)
                        qi += 1
                        continue
                    break
                active.append(a)
                qi += 1
            self.max_concurrent = max(self.max_concurrent, len(active))
            if not active:
                if qi < len(queue):
                    self.sleep(max(0.0, queue[qi].arrival_s - (self.clock() - t0)))
                continue
            self._round(active, out, t0)
            active = [a for a in active if "done" not in a]
        return out

    def _round(self, active: List[dict], out: List[Record], t0: float) -> None:
        """Advance the active solves (an engine step that returns 0 made no progress: the
        device is still busy, so the loop yields briefly); finished ones retire (marked
        "done")."""
        stepped = self.eng.step([a["h"] for a in active])
        self.rounds += 1
        for a in active:
            done, _ = self.eng.query(a["h"])
            if done:
                out.append(self._retire(a, self.clock() - t0))
                a["done"] = True
        if stepped == 0:
            self.sleep(self.cfg.poll_s)

    def _run_async(self, requests: Sequence, rhs_of: Callable[[Any], np.ndarray],
                   pool) -> List[Record]:
        queue = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        t0 = self.clock()
        active: List[dict] = []
        pending: List[dict] = []
        building: dict = {}
        out: List[Record] = []
        qi = 0
        while qi < len(queue) or active or pending:
            now = self.clock() - t0
            while (qi < len(queue) and queue[qi].arrival_s <= now
                   and len(active) + len(pending) < self.cfg.max_active):
                req = queue[qi]
                a = self._admit_async(req, rhs_of(req), self.clock() - t0, pool, building)
                if a is None:
                    if not active and not pending:
                        r = Record(req.rid, req.arrival_s, status=capi.NOMEM)
                        r.done_s = self.clock() - t0
                        out.append(r)
                        self.rejected.append(req.rid)
                        qi += 1
                        continue
                    break
                (pending if "build" in a else active).append(a)
                qi += 1
            self.max_concurrent = max(self.max_concurrent, len(active) + len(pending))
            if pending:
                if not active:
                    # nothing to step: wait for a build, or until the next arrival
                    timeout = None
                    if qi < len(queue):
                        timeout = max(0.0, queue[qi].arrival_s - (self.clock() - t0))
                    cf.wait({p["build"]["fut"] for p in pending}, timeout=timeout,
                            return_when=cf.FIRST_COMPLETED)
                ready = [p for p in pending if p["build"]["fut"].done()]
                for p in ready:
                    pending.remove(p)
                    active.append(self._start_pending(p, building))
            if not active:
                if not pending and qi < len(queue):
                    self.sleep(max(0.0, queue[qi].arrival_s - (self.clock() - t0)))
                continue
            self._round(active, out, t0)
            active = [a for a in active if "done" not in a]
        return out

    def close(self) -> None:
        for key in list(self.cache.keys()):
            self._drop(key)
        self.used = 0


def summarize(records: Sequence[Record]) -> Dict[str, float]:
    ok = [r for r in records if r.status == capi.OK]
    lat = np.array([r.latency_s for r in ok]) if ok else np.array([np.nan])
    t_first = min(r.arrival_s for r in records)
    t_last = max(r.done_s for r in records)
    span = max(t_last - t_first, 1e-9)
    return {
        "requests": len(records),
        "completed": len(ok),
        "rejected": sum(1 for r in records if r.status == capi.NOMEM),
        "solves_per_s": len(ok) / span,
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_iterations": float(np.mean([r.iterations for r in ok])) if ok else float("nan"),
        "dof_iter_per_s": sum(r.dof * r.iterations for r in ok) / span,
        "cache_hits": sum(1 for r in ok if r.cache_hit),
        "warm_starts": sum(1 for r in ok if r.warm_from >= 0),
        "mean_iterations_warm": (float(np.mean([r.iterations for r in ok if r.warm_from >= 0]))
                                 if any(r.warm_from >= 0 for r in ok) else float("nan")),
        "mean_iterations_cold": (float(np.mean([r.iterations for r in ok if r.warm_from < 0]))
                                 if any(r.warm_from < 0 for r in ok) else float("nan")),
        "max_rel_res": float(max((r.rel_res for r in ok), default=float("nan"))),
    }
