"""Continuous-batching request loop for many independent solves on one GPU.

Requests (grid side + seed) arrive over time.  A request is admitted as soon
as a worker slot is free and the device-memory footprint of everything in
flight plus its own stays within the budget; otherwise it waits in FIFO
order.  Each slot owns a HIP stream and keeps one solver hierarchy per grid
side resident on the device (created on first use, reused afterwards), so
admitted requests run concurrently and their kernels overlap.  A request's
work on its slot: draw its fields on the GPU, build the hierarchy for its
permeability (mscg_set_permeability), solve (mscg_solve).  Latency is
completion minus arrival; it includes queueing.

The solver itself is libmscg; this module only schedules.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

from . import mscg, synth


@dataclass
class Result:
    idx: int
    side: int
    arrival_s: float
    admit_s: float
    done_s: float
    slot: int
    status: int
    outer_iters: int
    rel_residual_true: float
    footprint: int
    solution: object = None  # device tensor, kept only for requests in `keep`
    error: str = ""

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


@dataclass
class ServeReport:
    results: list
    wall_s: float
    peak_inflight_bytes: int
    peak_inflight: int
    max_queue: int

    def summary(self) -> dict:
        import numpy as np
        lat = np.array([r.latency_s for r in self.results]) * 1e3
        ok = sum(1 for r in self.results if r.status == 0)
        return {
            "requests": len(self.results), "ok": ok, "wall_s": round(self.wall_s, 3),
            "solves_per_s": round(len(self.results) / self.wall_s, 2),
            "unknowns_per_s": round(sum(r.side * r.side for r in self.results) / self.wall_s, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "max_queue": self.max_queue,
            "peak_inflight": self.peak_inflight, "peak_inflight_bytes": self.peak_inflight_bytes,
            "max_rel_residual": max(r.rel_residual_true for r in self.results),
        }


class Server:
    def __init__(self, slots: int = 8, budget_bytes: int = 32 << 30, options: mscg.Options | None = None,
                 tol: float = 1e-8, device=None):
        import torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.options = options or mscg.Options(precision=mscg.MIXED)
        self.tol = tol
        self.budget = int(budget_bytes)
        self.nslots = slots
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.cache = [dict() for _ in range(slots)]  # side -> (Problem, p buffer)
        self._fp = {}

    def footprint(self, side: int) -> int:
        """Device bytes a request holds while in flight: hierarchy + k, f, p."""
        if side not in self._fp:
            grid = mscg.Grid(dim=2, n=(side, side))
            self._fp[side] = mscg.footprint_bytes(grid, self.options) + 3 * side * side * 8
        return self._fp[side]

    def _problem(self, slot: int, side: int):
        import torch
        c = self.cache[slot]
        if side not in c:
            with torch.cuda.stream(self.streams[slot]):
                grid = mscg.Grid(dim=2, n=(side, side))
                prob = mscg.Problem(grid, self.options, stream=self.streams[slot], device=self.device)
                c[side] = prob
        return c[side]

    def _run_one(self, slot: int, req: synth.Request, keep: bool):
        import torch
        stream = self.streams[slot]
        prob = self._problem(slot, req.side)
        with torch.cuda.stream(stream):
            k, f = synth.request_fields_torch(req, self.device, stream=stream)
            p = torch.zeros(req.side * req.side, dtype=torch.float64, device=self.device)
        prob.set_permeability(k, k)
        st = prob.solve(f, p, self.tol)
        return st, (p if keep else None)

    def run(self, requests, keep=(), time_scale: float = 1.0) -> ServeReport:
        """Serves `requests` (arrival times in seconds from the start, scaled by
        time_scale).  Returns per-request results in request order."""
        import torch
        keep = set(keep)
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        results = [None] * len(reqs)
        pos = {r.idx: i for i, r in enumerate(reqs)}
        lock = threading.Condition()
        pending = deque()
        free = list(range(self.nslots))
        work = [deque() for _ in range(self.nslots)]
        state = {"inflight_bytes": 0, "inflight": 0, "peak_bytes": 0, "peak": 0, "max_queue": 0, "done": 0,
                 "stop": False, "error": None}
        t0 = time.perf_counter()

        def worker(slot):
            torch.cuda.set_device(self.device)
            while True:
                with lock:
                    while not work[slot] and not state["stop"]:
                        lock.wait()
                    if not work[slot]:
                        return
                    req, admit_s = work[slot].popleft()
                err = ""
                try:
                    st, sol = self._run_one(slot, req, req.idx in keep)
                    status, outer, res = st.status, st.outer_iters, st.rel_residual_true
                    if status != 0:
                        err = mscg.last_error()  # thread-local, read on the worker's thread
                except Exception as e:  # a failing request does not stop the others
                    status, outer, res, sol = mscg.E_DEVICE, 0, float("inf"), None
                    err = repr(e)
                done_s = time.perf_counter() - t0
                fp = self.footprint(req.side)
                with lock:
                    results[pos[req.idx]] = Result(req.idx, req.side, req.arrival_s * time_scale, admit_s, done_s, slot,
                                                   status, outer, res, fp, sol, err)
                    state["inflight_bytes"] -= fp
                    state["inflight"] -= 1
                    state["done"] += 1
                    free.append(slot)
                    lock.notify_all()

        threads = [threading.Thread(target=worker, args=(s,), daemon=True) for s in range(self.nslots)]
        for t in threads:
            t.start()

        def admit_locked():
            while pending and free:
                req = pending[0]
                fp = self.footprint(req.side)
                if state["inflight"] > 0 and state["inflight_bytes"] + fp > self.budget:
                    break  # FIFO: wait for memory to free up
                pending.popleft()
                slot = free.pop()
                state["inflight_bytes"] += fp
                state["inflight"] += 1
                state["peak_bytes"] = max(state["peak_bytes"], state["inflight_bytes"])
                state["peak"] = max(state["peak"], state["inflight"])
                work[slot].append((req, time.perf_counter() - t0))
                lock.notify_all()

        i = 0
        with lock:
            while state["done"] < len(reqs):
                now = time.perf_counter() - t0
                while i < len(reqs) and reqs[i].arrival_s * time_scale <= now:
                    pending.append(reqs[i])
                    i += 1
                state["max_queue"] = max(state["max_queue"], len(pending))
                admit_locked()
                if state["done"] >= len(reqs):
                    break
                timeout = None
                if i < len(reqs):
                    timeout = max(0.0, reqs[i].arrival_s * time_scale - (time.perf_counter() - t0))
                lock.wait(timeout=timeout if timeout is not None else 0.05)
            state["stop"] = True
            lock.notify_all()
        for t in threads:
            t.join()
        wall = time.perf_counter() - t0
        torch.cuda.synchronize(self.device)
        return ServeReport(results=results, wall_s=wall, peak_inflight_bytes=state["peak_bytes"],
                           peak_inflight=state["peak"], max_queue=state["max_queue"])


def solve_alone(req: synth.Request, options: mscg.Options, tol: float = 1e-8, device=None):
    """The same request solved by itself on a fresh problem and stream."""
    import torch
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.Stream(device=device)
    with torch.cuda.stream(stream):
        prob = mscg.Problem(mscg.Grid(dim=2, n=(req.side, req.side)), options, stream=stream, device=device)
        k, f = synth.request_fields_torch(req, device, stream=stream)
        p = torch.zeros(req.side * req.side, dtype=torch.float64, device=device)
    prob.set_permeability(k, k)
    st = prob.solve(f, p, tol)
    torch.cuda.synchronize(device)
    return st, p, k, f
