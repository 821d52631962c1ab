"""Continuous-batching request loop for SRT forward and adjoint applies.

Plans (and their operator weights) stay resident on the device, one per grid
and aperture. Requests arrive over time, each naming a plan, a direction
(forward or adjoint) and a payload. The scheduler

  * admits a request only when the device memory it needs (its share of the
    batch input and output plus the batch workspace, srt_plan_footprint)
    fits in what the budget leaves after the work already in flight;
  * batches waiting requests that share a plan and a direction (oldest
    first, up to max_batch) into one batched apply -- the batch dimension
    only widens the dense operand of both CRT stages, so results are bitwise
    the same alone and batched;
  * keeps up to n_streams batches in flight on separate HIP streams, so work
    for different plans overlaps on the device, and admits new work as soon
    as a batch completes (no waiting for the queue to drain).

Latency of a request = completion time - arrival time (one clock for both).
The scheduler is pure host logic over an executor interface; GpuExecutor runs
applies through the C ABI, SimExecutor models durations for CPU tests.
"""
from __future__ import annotations

import dataclasses
import heapq
import time
from collections import deque
from typing import Any, Callable, Dict, List, Optional


@dataclasses.dataclass(eq=False)
class Request:
    rid: int
    plan: str                 # key of the plan in the server's plan table
    kind: str                 # "fwd" or "adj"
    payload: Any              # tensor (single item, no batch dimension)
    arrival: float            # seconds on the scheduler clock
    admit: Optional[float] = None
    finish: Optional[float] = None
    result: Any = None
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finish is None else self.finish - self.arrival


@dataclasses.dataclass(eq=False)
class Batch:
    plan: str
    kind: str
    reqs: List[Request]
    nbytes: int
    handle: Any = None        # executor's in-flight token


class Scheduler:
    """Admission by device-memory footprint plus continuous batching."""

    def __init__(self, footprint: Callable[[str, str, int], int], budget: int,
                 max_batch: int = 8, max_inflight: int = 4):
        self.footprint = footprint        # (plan, kind, batch) -> bytes
        self.budget = int(budget)
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight)
        self.waiting: deque = deque()
        self.inflight: List[Batch] = []
        self.in_use = 0
        self.peak_in_use = 0
        self.rejected: List[Request] = []

    def enqueue(self, r: Request):
        if self.footprint(r.plan, r.kind, 1) > self.budget:
            r.error = "request needs more device memory than the whole budget"
            self.rejected.append(r)
        else:
            self.waiting.append(r)

    def next_batch(self) -> Optional[Batch]:
        """The next batch to launch now, or None (no slot or no memory)."""
        if not self.waiting or len(self.inflight) >= self.max_inflight:
            return None
        head = self.waiting[0]
        same = [r for r in self.waiting if r.plan == head.plan and r.kind == head.kind]
        n = min(len(same), self.max_batch)
        while n > 0 and self.in_use + self.footprint(head.plan, head.kind, n) > self.budget:
            n -= 1
        if n == 0:
            return None
        chosen = same[:n]
        ids = {id(r) for r in chosen}
        self.waiting = deque(r for r in self.waiting if id(r) not in ids)
        b = Batch(head.plan, head.kind, chosen, self.footprint(head.plan, head.kind, n))
        self.in_use += b.nbytes
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.inflight.append(b)
        return b

    def complete(self, b: Batch):
        self.inflight.remove(b)
        self.in_use -= b.nbytes


class SimExecutor:
    """Executor for host-only tests: a batch of B items of plan p takes
    cost(p, kind, B) seconds of a virtual clock and runs on one of
    n_streams virtual streams (streams run concurrently)."""

    def __init__(self, cost: Callable[[str, str, int], float]):
        self.cost = cost
        self.now = 0.0
        self._done: list = []
        self._seq = 0

    def clock(self) -> float:
        return self.now

    def launch(self, b: Batch, now: float):
        self._seq += 1
        heapq.heappush(self._done, (now + self.cost(b.plan, b.kind, len(b.reqs)), self._seq, b))
        return self._seq

    def poll(self, now: float) -> List[Batch]:
        out = []
        while self._done and self._done[0][0] <= now:
            t, _, b = heapq.heappop(self._done)
            for r in b.reqs:
                r.finish = t
                r.result = ("done", r.rid)
            out.append(b)
        return out

    def next_event(self) -> Optional[float]:
        return self._done[0][0] if self._done else None

    def wait_until(self, t: float):
        self.now = max(self.now, t)


class GpuExecutor:
    """Runs batches through the C ABI on a pool of HIP streams (all at the
    default priority). Inputs are stacked into one device buffer per batch,
    the apply is launched on the batch's stream, and an event marks its end.
    A batch's stream first waits for the stream that was current when the
    batch was launched, so payloads written there are complete before they
    are read, and device payloads are marked as used on the batch's stream so
    that their memory is not reused while it reads them. At most n_streams
    batches can be in flight (the scheduler's max_inflight must not exceed
    it).

    With keep_results a finished request carries its output as a device
    tensor (a view of the batch output); without it the output is released
    at completion, as a server that has handed the result on would."""

    def __init__(self, plans: Dict[str, Any], n_streams: int = 4, keep_results: bool = True):
        import torch
        self.torch = torch
        self.plans = plans
        self.keep_results = keep_results
        self.n_streams = int(n_streams)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.free = list(range(n_streams))
        self.inflight: list = []
        self.t0 = time.perf_counter()

    def clock(self) -> float:
        return time.perf_counter() - self.t0

    def launch(self, b: Batch, now: float):
        torch = self.torch
        plan = self.plans[b.plan]
        if not self.free:
            raise RuntimeError("no free stream: more batches in flight than n_streams")
        si = self.free.pop()
        s = self.streams[si]
        s.wait_stream(torch.cuda.current_stream())
        for r in b.reqs:
            if r.payload.is_cuda:
                r.payload.record_stream(s)
        with torch.cuda.stream(s):
            x = torch.stack([r.payload.to("cuda", non_blocking=True) for r in b.reqs])
            # each batch gets its own workspace: batches of one plan may overlap
            ws = plan.workspace(len(b.reqs))
            if b.kind == "fwd":
                out = plan.forward(x, workspace=ws, stream=s)
            else:
                out = plan.adjoint(x, workspace=ws, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.inflight.append((b, ev, si, (x, ws), out))
        return ev

    def poll(self, now: float) -> List[Batch]:
        done = []
        keep = []
        for item in self.inflight:
            b, ev, si, x, out = item
            if ev.query():
                t = self.clock()
                for i, r in enumerate(b.reqs):
                    r.finish = t
                    r.result = out[i] if self.keep_results else None
                self.free.append(si)
                done.append(b)
            else:
                keep.append(item)
        self.inflight = keep
        return done

    def next_event(self) -> Optional[float]:
        return None

    # completions are found by polling events; a short sleep keeps the delay
    # between a batch ending and its requests finishing near the sleep's own
    # granularity on Linux (~50 us)
    POLL_S = 5e-5

    def wait_until(self, t: float):
        dt = t - self.clock()
        if dt > 0:
            time.sleep(min(dt, self.POLL_S))


def serve(trace: List[Request], sched: Scheduler, ex, realtime: bool = True) -> List[Request]:
    """Runs the arrival trace to completion. Requests become visible to the
    scheduler at their arrival time; batches launch as soon as admission
    allows and complete asynchronously."""
    if sched.max_inflight > getattr(ex, "n_streams", sched.max_inflight):
        raise ValueError("the scheduler's max_inflight exceeds the executor's streams")
    pending = sorted(trace, key=lambda r: r.arrival)
    i = 0
    n = len(pending)
    finished: List[Request] = []
    while len(finished) + len(sched.rejected) < n:
        now = ex.clock()
        while i < n and pending[i].arrival <= now:
            sched.enqueue(pending[i])
            i += 1
        for b in ex.poll(now):
            sched.complete(b)
            finished.extend(b.reqs)
        launched = False
        while True:
            b = sched.next_batch()
            if b is None:
                break
            for r in b.reqs:
                r.admit = now
            b.handle = ex.launch(b, now)
            launched = True
        if launched:
            continue
        if len(finished) + len(sched.rejected) >= n:
            break
        # nothing to launch: advance to the next arrival or completion
        nxt = [t for t in (pending[i].arrival if i < n else None, ex.next_event()) if t is not None]
        if nxt:
            ex.wait_until(min(nxt))
        elif realtime:
            ex.wait_until(now + 5e-5)
        else:
            raise RuntimeError("scheduler stalled with work left")
    return finished + sched.rejected


def latency_stats(reqs: List[Request]) -> dict:
    import numpy as np
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    if lat.size == 0:
        return {"n": 0}
    span = max(r.finish for r in reqs if r.finish is not None) - min(r.arrival for r in reqs)
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "throughput_rps": float(lat.size / span) if span > 0 else float("inf")}


def plan_footprint_fn(plans: Dict[str, Any]) -> Callable[[str, str, int], int]:
    """Device bytes a batch of B requests of a plan needs while in flight:
    stacked input, output and the plan's workspace for B items (FP32 or FP64
    values per the plan)."""
    def fp(key: str, kind: str, b: int) -> int:
        p = plans[key]
        esz = 8 if p.value_dtype == "f64" else 4
        vol = p.mz * p.ms * p.ms * esz
        dat = p.n_angles * p.n_z * p.n_radii * esz
        return b * (vol + dat) + p.footprint(b)[1]
    return fp
