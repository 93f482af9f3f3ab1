"""Ad-hoc layer pricing with continuous batching (the real-time pricing use of
section 1: an underwriter prices a contract while on the phone with a client).

The YET stays resident in HBM.  Requests (a layer of XELTs and terms, a seed
and a program id chosen by the client) are admitted while their tables fit
the HBM budget; admitted requests share every launch.  A global cursor walks
the YET in trial tiles; each tick evaluates the current tile for every active
request in one ``ara_run_prepared`` launch, so a request that arrives while
others are on the GPU joins at the next tile boundary and overlaps with them.
A request is complete once the cursor has covered all N trials since it
joined (wrapping around); its PML/TVaR are then computed on the device and
its memory released for waiting requests.  Each trial's year loss depends only
on the trial, the layer and the request's seed, so a result is the same alone
and in any mix.  A request can be cancelled, or given a deadline after its
arrival: either way it leaves the server with its memory released and no
result, and the others are unaffected.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import (ARA_E_BUDGET, DEFAULT_RETURN_PERIODS, AraError, ara_free_elts, ara_free_layer, ara_load_elts,
               ara_prepare_layer, ara_risk_measures, ara_run_prepared, layer_desc)


@dataclass
class Request:
    req_id: int
    layer: object                 # synth.Layer-like: elts, terms, program_id
    seed: int
    arrival: float = 0.0          # seconds since the start of the run
    deadline: float = math.inf    # seconds after arrival; past it the request is dropped
    # filled by the server
    status: str = "waiting"       # waiting, active, done, cancelled or timed_out
    elt_handles: List[int] = field(default_factory=list)
    prepared: int = -1
    ylt: object = None            # torch tensor [N] on the device
    start: int = 0                # cursor value at admission
    done: int = 0                 # trials evaluated so far
    admitted_at: float = math.nan
    finished_at: float = math.nan
    pml: Optional[np.ndarray] = None
    tvar: Optional[np.ndarray] = None
    bytes: int = 0

    @property
    def latency(self) -> float:
        return self.finished_at - self.arrival


def request_bytes(layer, catalog_size: int, n_trials: int, mode: int) -> int:
    """Device bytes a request holds while active (XELT tables, layer tables, YLT)."""
    n = sum(e.n for e in layer.elts)
    elts = len(layer.elts) * catalog_size * 4 + n * (32 + 8)
    tables = catalog_size * (16 + 8) + (catalog_size // 1024 + 1) * 4 + n * (32 + (16 if mode == 2 else 0))
    return int(elts + tables + n_trials * 4 + 4096)


class PricingServer:
    def __init__(self, engine, yet_handle: int, n_trials: int, events_per_trial: int, catalog_size: int,
                 mode: int, hbm_budget_bytes: int, tile: int = 65536,
                 return_periods: Sequence[float] = DEFAULT_RETURN_PERIODS, max_active: int = 128,
                 max_inflight: int = 2):
        import torch
        self.torch = torch
        self.eng = engine
        self.ctx = engine.ctx
        self.yet = yet_handle
        self.N = int(n_trials)
        self.K = int(events_per_trial)
        self.C = int(catalog_size)
        self.mode = int(mode)
        self.budget = int(hbm_budget_bytes)
        self.tile = int(tile)
        self.rps = tuple(return_periods)
        self.max_active = int(max_active)
        self.max_inflight = max(1, int(max_inflight))
        self.inflight: collections.deque = collections.deque()     # one event per queued tick
        self.cursor = 0
        self.used = 0
        self.waiting: collections.deque = collections.deque()
        self.active: List[Request] = []
        self.finished: List[Request] = []
        self.dropped: List[Request] = []            # cancelled or timed out
        self.refusals = 0
        self.ticks = 0
        self.t0 = time.perf_counter()

    # ------------------------------------------------------------ admission
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        req.status = "waiting"
        self.waiting.append(req)

    def cancel(self, req_id: int, status: str = "cancelled") -> bool:
        """Drop a waiting or active request: its layer tables and YLT are
        released at once (work already queued for it completes first on the
        device, ordered by the library), and it finishes with no result."""
        for r in list(self.waiting):
            if r.req_id == req_id:
                self.waiting.remove(r)
                self._drop(r, status)
                return True
        for r in self.active:
            if r.req_id == req_id:
                self.active.remove(r)
                ara_free_layer(self.ctx, r.prepared)
                r.prepared = -1
                self.used -= r.bytes
                r.ylt = None
                self._drop(r, status)
                return True
        return False

    def _drop(self, r: Request, status: str) -> None:
        r.status = status
        r.finished_at = self.now()
        self.dropped.append(r)

    def _expire(self) -> None:
        now = self.now()
        for r in [r for r in list(self.waiting) + self.active if now > r.arrival + r.deadline]:
            self.cancel(r.req_id, status="timed_out")

    def _admit(self) -> None:
        while self.waiting and len(self.active) < self.max_active:
            req = self.waiting[0]
            need = request_bytes(req.layer, self.C, self.N, self.mode)
            if need > self.budget:
                self.waiting.popleft()
                raise AraError(ARA_E_BUDGET, f"request {req.req_id} needs {need} bytes, more than the whole budget")
            if self.used + need > self.budget:
                self.refusals += 1
                return                       # wait for memory to free up (FIFO)
            try:
                req.elt_handles = ara_load_elts(self.ctx, self.C, req.layer.elts)
                desc = layer_desc(req.elt_handles, req.layer.occ_retention, req.layer.occ_limit,
                                  req.layer.agg_retention, req.layer.agg_limit, req.layer.program_id)
                req.prepared = ara_prepare_layer(self.ctx, desc, self.mode)
            except AraError as e:
                if e.status != ARA_E_BUDGET:
                    raise
                if req.elt_handles:
                    ara_free_elts(self.ctx, req.elt_handles)
                    req.elt_handles = []
                self.refusals += 1
                return
            # the layer tables are self-contained: the XELTs can go
            ara_free_elts(self.ctx, req.elt_handles)
            req.elt_handles = []
            req.ylt = self.torch.empty(self.N, dtype=self.torch.float32, device="cuda")
            req.bytes = need
            req.start = self.cursor
            req.done = 0
            req.admitted_at = self.now()
            req.status = "active"
            self.used += need
            self.waiting.popleft()
            self.active.append(req)

    # ------------------------------------------------------------ one tick
    def tick(self) -> None:
        """Drop what is past its deadline, admit what fits, then evaluate the
        current trial tile for every active request in one launch."""
        self._expire()
        self._admit()
        if not self.active:
            return
        t0 = self.cursor
        t1 = min(self.N, t0 + self.tile)
        # a request never evaluates past its own N trials
        reqs = [r for r in self.active if r.done < self.N]
        handles = [r.prepared for r in reqs]
        seeds = [r.seed for r in reqs]
        outs = [r.ylt.data_ptr() + 4 * t0 for r in reqs]
        stream = self.torch.cuda.current_stream()
        ara_run_prepared(self.ctx, self.yet, handles, seeds, t0, t1, outs, stream=stream.cuda_stream)
        ev = self.torch.cuda.Event()
        ev.record(stream)
        self.inflight.append(ev)
        # Bounded run-ahead: the host queues at most max_inflight ticks, so a
        # request that arrives now starts within that many tiles instead of
        # behind a whole wrap of queued tiles.
        while len(self.inflight) > self.max_inflight:
            self.inflight.popleft().synchronize()
        for r in reqs:
            r.done += t1 - t0
        self.cursor = 0 if t1 >= self.N else t1
        self.ticks += 1
        for r in [r for r in self.active if r.done >= self.N]:
            self._finish(r)

    def _finish(self, r: Request) -> None:
        pml, tvar = ara_risk_measures(self.ctx, r.ylt, self.rps)    # waits for the request's last tile
        self.inflight.clear()                                         # ... and every tick before it
        r.pml, r.tvar = pml, tvar
        r.status = "done"
        r.finished_at = self.now()
        ara_free_layer(self.ctx, r.prepared)
        self.used -= r.bytes
        self.active.remove(r)
        self.finished.append(r)

    # ------------------------------------------------------------ drivers
    def run_open_loop(self, requests: Sequence[Request], keep_ylt: bool = False) -> List[Request]:
        """Serve requests arriving at their `arrival` times (seconds from now)."""
        pending = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        i = 0
        while i < len(pending) or self.waiting or self.active:
            now = self.now()
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            if self.waiting or self.active:
                self.tick()
            elif i < len(pending):
                time.sleep(max(0.0, min(0.002, pending[i].arrival - self.now())))
        self.torch.cuda.synchronize()
        if not keep_ylt:
            for r in self.finished:
                r.ylt = None
        return self.finished


def poisson_arrivals(rate: float, n: int, seed: int = 1310) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def latency_stats(reqs: Sequence[Request]) -> Dict[str, float]:
    lat = np.array([r.latency for r in reqs])
    return {"n": int(lat.size), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}
