"""Host-only tests of the serving scheduler (admission by device-memory
footprint, continuous batching) on a simulated executor with a virtual clock."""
import numpy as np

from paper_2402_15641_amd.serve import (Request, Scheduler, SimExecutor, latency_stats,
                                        serve)

MB = 1 << 20
SIZES = {"s64": 4 * MB, "s128": 32 * MB, "s192": 100 * MB}     # bytes per item
WS = {"s64": 40 * MB, "s128": 300 * MB, "s192": 900 * MB}      # workspace per item
COST = {"s64": 0.2e-3, "s128": 1.5e-3, "s192": 5e-3}            # seconds per item


def footprint(plan, kind, b):
    return b * (SIZES[plan] + WS[plan])


def cost(plan, kind, b):
    return COST[plan] * (0.4 + 0.6 * b)  # batching amortises a fixed part


def trace(n, rate, seed=0, plans=("s64", "s128", "s192")):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    return [Request(i, plans[rng.integers(len(plans))], "fwd" if rng.random() < 0.7 else "adj",
                    None, float(t[i])) for i in range(n)]


class RecordingExecutor(SimExecutor):
    def __init__(self, cost):
        super().__init__(cost)
        self.batch_sizes = []

    def launch(self, b, now):
        self.batch_sizes.append(len(b.reqs))
        return super().launch(b, now)


def run(reqs, budget, max_batch=8, max_inflight=4, ex=None):
    sched = Scheduler(footprint, budget, max_batch, max_inflight)
    done = serve(reqs, sched, ex or SimExecutor(cost), realtime=False)
    return sched, done


def test_every_request_finishes_within_budget():
    reqs = trace(500, 400.0)
    sched, done = run(reqs, budget=4 << 30)
    assert len(done) == 500 and not sched.rejected
    assert all(r.finish >= r.admit >= r.arrival for r in done)
    assert sched.peak_in_use <= 4 << 30
    assert sched.in_use == 0 and not sched.inflight


def test_batches_group_same_plan_and_direction():
    reqs = [Request(i, "s64", "fwd", None, 0.0) for i in range(20)]
    reqs += [Request(100 + i, "s64", "adj", None, 0.0) for i in range(3)]
    ex = RecordingExecutor(cost)
    sched, done = run(reqs, budget=16 << 30, max_batch=8, ex=ex)
    # 20 simultaneous forwards -> 8, 8, 4; the 3 adjoints form their own batch
    assert sorted(ex.batch_sizes) == [3, 4, 8, 8]
    assert len(done) == 23


def test_tiny_budget_serialises_but_completes():
    reqs = trace(60, 1000.0, seed=1)
    budget = footprint("s192", "fwd", 1)  # exactly one large item at a time
    sched, done = run(reqs, budget=budget)
    assert len(done) == 60 and not sched.rejected
    assert sched.peak_in_use <= budget


def test_oversized_request_is_rejected_not_fatal():
    reqs = trace(30, 500.0, seed=2, plans=("s64",))
    reqs.append(Request(999, "s192", "fwd", None, 0.01))
    sched, done = run(reqs, budget=footprint("s192", "fwd", 1) - 1)
    bad = [r for r in done if r.rid == 999][0]
    assert bad.error and bad.finish is None
    assert sum(1 for r in done if r.finish is not None) == 30


def test_continuous_admission_overlaps_inflight_work():
    """A request arriving while a long batch runs is admitted (and finishes)
    before that batch completes: admission does not wait for the queue."""
    reqs = [Request(0, "s192", "fwd", None, 0.0), Request(1, "s64", "adj", None, 0.001)]
    sched, done = run(reqs, budget=16 << 30)
    big = [r for r in done if r.rid == 0][0]
    small = [r for r in done if r.rid == 1][0]
    assert small.admit < big.finish and small.finish < big.finish


def test_latency_stats_and_throughput_grow_with_rate():
    lo = latency_stats(run(trace(400, 100.0, seed=3), budget=8 << 30)[1])
    hi = latency_stats(run(trace(400, 2000.0, seed=3), budget=8 << 30)[1])
    assert lo["n"] == hi["n"] == 400
    assert hi["throughput_rps"] > lo["throughput_rps"]
    assert lo["p99_ms"] >= lo["p50_ms"] > 0


def test_deterministic():
    a = run(trace(200, 800.0, seed=4), budget=2 << 30)[1]
    b = run(trace(200, 800.0, seed=4), budget=2 << 30)[1]
    assert [(r.rid, r.admit, r.finish) for r in a] == [(r.rid, r.admit, r.finish) for r in b]
