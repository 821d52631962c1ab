"""Serving benchmark: p50/p99 latency and throughput of a mixed request stream.

Workload: grids drawn uniformly from 64^3, 128^3 and 192^3 on [-1,1]^3,
apertures N columns x N heights x 4N radii on a cylinder of radius 1.3
(l_max = distance to the farthest voxel corner); 70% forward requests
(ellipsoid phantoms, 16 per grid, seeded) and 30% adjoint requests (N(0,1)
data, 16 per grid); Poisson arrivals at each rate (the two highest default
rates exceed what one GPU serves, so there the throughput is the capacity);
plans resident on the device; admission by device-memory footprint (default budget 16 GiB);
continuous batching (up to 8 per batch) on 4 streams. Run once with FP32
operator weights and once with BF16 weights (FP32 accumulation).

    python -m paper_2402_15641_amd.serve_bench [--rates 50 100 ...] [--weights f32 bf16]

Prints one JSON line per (weights, rate).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np


def serving_mix(rates, weights=("f32", "bf16"), seconds=1.0, min_requests=5000,
                budget_gib=16.0, sizes=(64, 128, 192), pool=16, log=None):
    """Runs the mixed request stream at each rate for each weight type and
    returns the records: per weight type one capacity record (device time
    per request in batches of 8), then one latency record per rate. Plans
    and payloads are built here and released at the end."""
    import torch
    from srt_inputs import config, phantoms
    from paper_2402_15641_amd import SRTPlan
    from paper_2402_15641_amd.serve import (GpuExecutor, Request, Scheduler, latency_stats,
                                            plan_footprint_fn, serve)

    out = []
    emit = (lambda rec: (out.append(rec), log(rec) if log else None))
    pools = {}
    aps = {n: config(f"serve{n}") for n in sizes}
    for n, a in aps.items():
        vols = [torch.from_numpy(phantoms.ellipsoid_phantom(a, np.random.default_rng(5000 + 100 * n + i),
                                                            noise_rng=np.random.default_rng(6000 + 100 * n + i))
                                 ).float().cuda() for i in range(pool)]
        dats = [torch.from_numpy(np.random.default_rng(7000 + 100 * n + i).standard_normal(a.data_shape)
                                 ).float().cuda() for i in range(pool)]
        pools[n] = (vols, dats)
    for w in weights:
        plans = {f"n{n}": SRTPlan.from_geometry(a, value_dtype="f32", weight_dtype=w)
                 for n, a in aps.items()}
        fp = plan_footprint_fn(plans)
        # warm up every (plan, direction, batch size) once
        for key, p in plans.items():
            n = int(key[1:])
            for b in range(1, 9):
                p.forward(torch.stack([pools[n][0][i % pool] for i in range(b)]))
                p.adjoint(torch.stack([pools[n][1][i % pool] for i in range(b)]))
        torch.cuda.synchronize()
        # device time per request in full batches of 8, and the request rate
        # one GPU sustains on this mix when it does nothing else
        per_req = {}
        for key, p in plans.items():
            n = int(key[1:])
            for kind, pl, fn in (("fwd", pools[n][0], p.forward), ("adj", pools[n][1], p.adjoint)):
                x = torch.stack([pl[i % pool] for i in range(8)])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(5):
                    fn(x)
                e1.record()
                torch.cuda.synchronize()
                per_req[f"{key}_{kind}"] = e0.elapsed_time(e1) / 5 / 8
        mix_ms = sum((0.7 if k.endswith("fwd") else 0.3) / len(plans) * v for k, v in per_req.items())
        emit({"weights": w, "device_ms_per_request_batch8": per_req,
              "device_bound_capacity_rps": 1000.0 / mix_ms})
        for rate in rates:
            rng = np.random.default_rng(int(rate) + (0 if w == "f32" else 1))
            nreq = int(max(min_requests, rate * seconds))
            t = np.cumsum(rng.exponential(1.0 / rate, nreq))
            reqs = []
            for i in range(nreq):
                n = sizes[rng.integers(len(sizes))]
                kind = "fwd" if rng.random() < 0.7 else "adj"
                payload = pools[n][0 if kind == "fwd" else 1][rng.integers(pool)]
                reqs.append(Request(i, f"n{n}", kind, payload, float(t[i])))
            sched = Scheduler(fp, int(budget_gib * (1 << 30)), max_batch=8, max_inflight=4)
            # outputs are released at completion (handed on to the client)
            ex = GpuExecutor(plans, n_streams=4, keep_results=False)
            done = serve(reqs, sched, ex)
            torch.cuda.synchronize()
            st = latency_stats(done)
            st.update({"weights": w, "rate_rps": rate, "requests": nreq,
                       "peak_in_use_gib": sched.peak_in_use / (1 << 30),
                       "rejected": len(sched.rejected)})
            emit(st)
        for p in plans.values():
            p.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", type=float, nargs="+", default=[50, 100, 200, 500, 1000, 2000, 5000, 10000])
    ap.add_argument("--weights", nargs="+", default=["f32", "bf16"])
    ap.add_argument("--min-requests", type=int, default=5000)
    ap.add_argument("--seconds", type=float, default=1.0,
                    help="trace length per rate is max(min_requests, rate * seconds)")
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--sizes", type=int, nargs="+", default=[64, 128, 192])
    args = ap.parse_args()

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    serving_mix(args.rates, args.weights, args.seconds, args.min_requests, args.budget_gib,
                args.sizes, log=lambda rec: print(json.dumps(rec), flush=True))


if __name__ == "__main__":
    main()
