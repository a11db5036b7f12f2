"""A sequence of related Poisson solves, one per time step of a simulation (Section 5.2).

The paper compares three ways of constructing the preconditioner of each step:

* ``"rebuild"``: a new SA-AMG hierarchy every step (its default variant);
* ``"hierarchy"``: reusing the aggregation hierarchy -- the aggregates and tentative
  prolongators stay, every number is recomputed for the step's geometry (saamg_refresh);
* ``"preconditioner"``: reusing the preconditioner -- the one built at the first step serves
  the later steps while the system operator follows the geometry (saamg_set_operator), and
  it is rebuilt for the next step's geometry (saamg_refresh) once a solve needs more than
  ``max_iterations`` iterations, or more than ``growth`` times the iterations of the first
  solve after the last (re)build (either limit may be None).

Every solve starts from the previous step's solution (Section 4).  This module holds only
the policy; every numerical step runs in the library.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

from . import capi

MODES = ("rebuild", "hierarchy", "preconditioner")


@dataclasses.dataclass
class StepRecord:
    step: int
    iterations: int
    status: int
    rel_res: float
    rebuilt: bool      # the preconditioner was built for this step's geometry before its solve
    prec_ms: float     # host wall time of the preconditioner's construction or update
    solve_ms: float
    trigger: bool      # the solve exceeded the threshold: the next step rebuilds


class SolveSequence:
    """Solves A_k x_k = b_k for a sequence of domains with the same unknowns."""

    def __init__(self, variant: int, options: Optional[capi.Options] = None,
                 mode: str = "preconditioner", max_iterations: Optional[int] = None,
                 growth: Optional[float] = 1.5, tol: float = 1e-8, max_iter: int = 500,
                 device: int = 0):
        if mode not in MODES:
            raise ValueError(f"mode must be one of {MODES}")
        import torch
        self.torch = torch
        self.dev = torch.device(f"cuda:{device}")
        self.variant = variant
        self.options = options if options is not None else capi.default_options()
        self.mode = mode
        self.max_iterations = max_iterations
        self.growth = growth
        self.tol = tol
        self.max_iter = max_iter
        self.H: Optional[capi.Hierarchy] = None
        self.x = None          # previous solution (device, unscaled)
        self.base_it: Optional[int] = None
        self.stale = False     # the threshold was exceeded: rebuild at the next step
        self.records: List[StepRecord] = []

    def step(self, dom: capi.HostDomain, b) -> StepRecord:
        """One time step: the preconditioner for ``dom`` by the sequence's mode, then a
        warm-started solve of A x = b (b: device float64 box vector)."""
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        rebuilt = False
        if self.H is None or self.mode == "rebuild":
            if self.H is not None:
                capi.destroy(self.H)
            self.H = capi.setup(dom, self.variant, self.options)
            rebuilt = True
        elif self.mode == "hierarchy" or self.stale:
            capi.refresh(self.H, dom)
            rebuilt = True
        else:
            capi.set_operator(self.H, dom)
        torch.cuda.synchronize(self.dev)
        t1 = time.perf_counter()
        if rebuilt:
            self.base_it = None
            self.stale = False
        x = torch.zeros(self.H.nbox, dtype=torch.float64, device=self.dev)
        res = capi.solve(self.H, b, x, x0=self.x, tol=self.tol, max_iter=self.max_iter)
        torch.cuda.synchronize(self.dev)
        t2 = time.perf_counter()
        it = res["iterations"]
        if self.base_it is None:
            self.base_it = it
        trigger = self.mode == "preconditioner" and (
            (self.max_iterations is not None and it > self.max_iterations)
            or (self.growth is not None and it > self.growth * self.base_it))
        self.stale = trigger
        self.x = x
        rec = StepRecord(len(self.records), it, res["status"], res["rel_res_true"], rebuilt,
                         1e3 * (t1 - t0), 1e3 * (t2 - t1), trigger)
        self.records.append(rec)
        return rec

    def close(self) -> None:
        if self.H is not None:
            capi.destroy(self.H)
            self.H = None
