"""Continuous-batching serving loop for HEOM solves of different sizes.

Requests (a system, a hierarchy depth, an initial state and a number of RK4
steps) arrive over time.  The engine admits a waiting request as soon as its
device memory fits in the HBM budget, keeps its state on the device in a
workspace of its own for its whole life, and advances every admitted request
together: each engine iteration is one batched launch sequence over all active
requests (``heom_advance_slots``), so requests that arrive while others run
share the GPU with them.  A request leaves when its steps are done; only its
final reduced density matrix and sink populations are copied to the host.

The device work is behind a small backend interface (``admit``, ``advance``,
``release``); ``GpuBackend`` implements it with the HIP library.  Tests drive
the engine with a backend of their own and a virtual clock.  ``advance``
reports a failure per request; a request that failed leaves the engine, and
no request is ever advanced twice in one iteration.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import Callable, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    id: int
    system: dict
    depth: int
    rho0: np.ndarray
    steps: int
    dt: float = 1.0
    arrival_s: float = 0.0
    precision: str = "fp64"
    # filled by the engine
    status: str = "new"          # new, waiting, running, done, failed, rejected, cancelled
    admit_s: float = math.nan
    finish_s: float = math.nan
    steps_done: int = 0
    rho_final: Optional[np.ndarray] = None
    sinks: Optional[np.ndarray] = None   # P_trap, P_recomb, Q
    error: str = ""
    n_ados: int = 0

    @property
    def latency_s(self) -> float:
        return self.finish_s - self.arrival_s

    @property
    def eta(self) -> float:
        return float(self.sinks[0]) if self.sinks is not None else math.nan


class GpuBackend:
    """Device side of the engine on the HIP library (one GPU)."""

    def __init__(self, device: str = "cuda", stream=None, kernel: str = "auto"):
        import torch

        from . import heom

        self._torch = torch
        self._heom = heom
        self.device = device
        self.stream = stream
        self.kernel = kernel
        self._scratch = None

    def footprint(self, req: Request) -> tuple:
        """(bytes of device memory the request needs, built hierarchy)."""
        h = self._heom.Hierarchy(req.system, req.depth)
        prec = self._heom.PRECISIONS[req.precision]
        return h.workspace_bytes[prec] + tables_bytes(h), h

    def admit(self, req: Request, prepared) -> dict:
        h = prepared
        prec = self._heom.PRECISIONS[req.precision]
        ws = self._heom.allocate_workspace(h.workspace_bytes[prec], device=self.device)
        req.n_ados = h.n_ados
        return {"h": h, "ws": ws, "started": False}

    def advance(self, reqs, slots, n_steps: int):
        """Advances all slots by n_steps.  Returns (rho list, sinks array,
        error list) in order: error[i] is None, or the reason slot i failed
        (its state is then not to be continued)."""
        n = len(reqs)
        out_rho, out_sinks, errors = [None] * n, np.zeros((n, 3)), [None] * n
        # One launch sequence per precision and time step.
        by_prec = {}
        for i, r in enumerate(reqs):
            by_prec.setdefault((r.precision, r.dt), []).append(i)
        for (prec, _dt), idx in by_prec.items():
            hs = [slots[i]["h"] for i in idx]
            try:
                need = self._heom.slots_scratch_bytes(hs)
                if self._scratch is None or self._scratch.numel() < need:
                    self._scratch = self._heom.allocate_workspace(max(need, 1 << 20),
                                                                  device=self.device)
                rhos, sinks = self._heom.advance_slots(
                    hs, [slots[i]["ws"] for i in idx], [not slots[i]["started"] for i in idx],
                    [reqs[i].rho0 for i in idx], reqs[idx[0]].dt, n_steps, self._scratch,
                    precision=prec, stream=self.stream, kernel=self.kernel)
                failed = set()
            except self._heom.SlotsNumericError as e:
                # Every slot of the call advanced; only the non-finite ones failed.
                rhos, sinks, failed = e.rhos, e.sinks, set(e.failed)
                for j in failed:
                    errors[idx[j]] = f"non-finite result after {n_steps} more steps"
            except Exception as e:  # the state of every slot of this call is unknown
                for i in idx:
                    errors[i] = str(e)
                continue
            for j, i in enumerate(idx):
                slots[i]["started"] = True
                if j not in failed:
                    out_rho[i] = rhos[j]
                    out_sinks[i] = sinks[j]
        return out_rho, out_sinks, errors

    def release(self, slot) -> None:
        slot["ws"] = None
        slot["h"].close()


def tables_bytes(h) -> int:
    """Device bytes of the neighbour tables of a hierarchy, at most: two int32
    tables, the uint8 occupations and, where every neighbour lies within
    32767 ADOs, the two tables again as int16 offsets ([modes][ADOs padded to
    64])."""
    stride = (h.n_ados + 63) // 64 * 64
    return h.n_modes * stride * 13


class Engine:
    """Admission by HBM budget, continuous batching, latency bookkeeping.

    ``clock`` returns seconds; ``sleep`` waits for the next arrival when the
    GPU is idle.  ``chunk_steps`` bounds the RK4 steps of one iteration, so
    that new arrivals wait at most one iteration before they join.
    """

    def __init__(self, backend, hbm_budget_bytes: int, chunk_steps: int = 200,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, max_active: Optional[int] = None):
        if hbm_budget_bytes <= 0:
            raise ValueError("hbm_budget_bytes must be positive")
        if chunk_steps < 1:
            raise ValueError("chunk_steps must be >= 1")
        if max_active is not None and max_active < 1:
            raise ValueError("max_active must be >= 1")
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.chunk_steps = int(chunk_steps)
        self.max_active = max_active  # None: as many as the budget admits
        self.clock = clock
        self.sleep = sleep
        self.waiting: deque = deque()
        self.active: list = []   # (request, slot, bytes)
        self.finished: list = []
        self.in_use = 0
        self.iterations = 0
        self.occupancy_sum = 0
        self.ado_steps = 0
        self.t0 = None

    # -- request lifecycle ------------------------------------------------------

    def submit(self, req: Request) -> None:
        try:
            nbytes, prepared = self.backend.footprint(req)
        except Exception as e:  # invalid request: reject it alone
            req.status, req.error = "rejected", str(e)
            req.finish_s = self._now()
            self.finished.append(req)
            return
        if nbytes > self.budget:
            req.status = "rejected"
            req.error = f"needs {nbytes} bytes, budget is {self.budget}"
            req.finish_s = self._now()
            self.finished.append(req)
            return
        req.status = "waiting"
        self.waiting.append((req, nbytes, prepared))

    def cancel(self, req_id: int) -> bool:
        for k, (r, nb, prep) in enumerate(self.waiting):
            if r.id == req_id:
                del self.waiting[k]
                r.status, r.finish_s = "cancelled", self._now()
                self.finished.append(r)
                return True
        for k, (r, slot, nb) in enumerate(self.active):
            if r.id == req_id:
                del self.active[k]
                self._free(slot, nb)
                r.status, r.finish_s = "cancelled", self._now()
                self.finished.append(r)
                return True
        return False

    def _now(self) -> float:
        if self.t0 is None:
            self.t0 = self.clock()
        return self.clock() - self.t0

    def _free(self, slot, nbytes) -> None:
        self.backend.release(slot)
        self.in_use -= nbytes

    def _admit(self) -> None:
        # First come, first served: the head of the queue waits for memory; a
        # smaller request behind it does not overtake it.
        while (self.waiting and self.in_use + self.waiting[0][1] <= self.budget and
               (self.max_active is None or len(self.active) < self.max_active)):
            req, nbytes, prepared = self.waiting.popleft()
            try:
                slot = self.backend.admit(req, prepared)
            except Exception as e:
                req.status, req.error, req.finish_s = "failed", str(e), self._now()
                self.finished.append(req)
                continue
            self.in_use += nbytes
            req.status, req.admit_s = "running", self._now()
            self.active.append((req, slot, nbytes))

    # -- engine iteration -----------------------------------------------------------

    def step(self) -> bool:
        """One iteration: admit, advance all active requests, retire finished
        ones.  Returns False when there was nothing to run."""
        self._admit()
        if not self.active:
            return False
        k = min(self.chunk_steps, min(r.steps - r.steps_done for r, _, _ in self.active))
        reqs = [r for r, _, _ in self.active]
        slots = [s for _, s, _ in self.active]
        n = len(reqs)
        if k > 0:
            try:
                rhos, sinks, errors = self.backend.advance(reqs, slots, k)
            except Exception as e:
                # The backend cannot say which requests advanced: none of them
                # can be continued (re-running them could advance some twice).
                rhos, sinks, errors = [None] * n, np.zeros((n, 3)), [str(e)] * n
        else:
            rhos, sinks, errors = [None] * n, np.zeros((n, 3)), [None] * n
        # Failed requests leave the engine; every other one advanced by k.
        keep = []
        for i, (r, s, nb) in enumerate(self.active):
            if errors[i] is None:
                keep.append(i)
                continue
            r.status, r.error, r.finish_s = "failed", str(errors[i]), self._now()
            self.finished.append(r)
            self._free(s, nb)
        self.active = [self.active[i] for i in keep]
        rhos = [rhos[i] for i in keep]
        sinks = sinks[keep]
        self.iterations += 1
        self.occupancy_sum += len(self.active)
        still = []
        for i, (r, s, nb) in enumerate(self.active):
            r.steps_done += k
            self.ado_steps += r.n_ados * k
            r.rho_final, r.sinks = rhos[i], sinks[i]
            if r.steps_done >= r.steps:
                r.status, r.finish_s = "done", self._now()
                self.finished.append(r)
                self._free(s, nb)
            else:
                still.append((r, s, nb))
        self.active = still
        return True

    def run(self, requests, on_finish: Optional[Callable[[Request], None]] = None) -> dict:
        """Serves `requests` (sorted by arrival_s, seconds from the start) and
        returns the metrics.  ``on_finish`` is called with each request that
        leaves the engine (done, failed or rejected), in order."""
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        self._now()
        reported = len(self.finished)
        while pending or self.waiting or self.active:
            now = self._now()
            while pending and pending[0].arrival_s <= now:
                self.submit(pending.popleft())
            ran = self.step()
            if on_finish is not None:
                for r in self.finished[reported:]:
                    on_finish(r)
                reported = len(self.finished)
            if not ran and pending:
                self.sleep(max(0.0, pending[0].arrival_s - self._now()))
        return self.metrics()

    def metrics(self) -> dict:
        done = [r for r in self.finished if r.status == "done"]
        lat = np.array([r.latency_s for r in done]) if done else np.zeros(0)
        span = max((r.finish_s for r in self.finished), default=0.0)
        return {
            "completed": len(done),
            "rejected": sum(r.status == "rejected" for r in self.finished),
            "failed": sum(r.status == "failed" for r in self.finished),
            "cancelled": sum(r.status == "cancelled" for r in self.finished),
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else math.nan,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else math.nan,
            "makespan_s": span,
            "solves_per_s": len(done) / span if span > 0 else math.nan,
            "ado_steps_per_s": self.ado_steps / span if span > 0 else math.nan,
            "mean_occupancy": self.occupancy_sum / self.iterations if self.iterations else 0.0,
            "iterations": self.iterations,
        }
