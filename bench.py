#!/usr/bin/env python3
"""Benchmark: spherical Radon transform forward+adjoint pairs per second.

Workload (default): the PACT-scale cylindrical aperture -- 256^3 voxels at
0.1 mm, cylinder radius 15.36 mm, 512 columns x 256 heights x 1024 radii,
FP32 values, batch 1, phantom of 200 random thin cylinders (seeded). One step
is one srt_forward followed by one srt_adjoint of its result, with the plan,
the input volume and a caller workspace already resident in HBM.

Prints one JSON line on stdout. Besides throughput it reports:
  roofline      the dominant kernel's algorithmic FLOP rate, timed live with
                HIP events recorded by the library on the apply stream, against
                the FP32 vector-ALU peak (157.3 TFLOP/s; gfx950 issues unpacked
                v_fmac_f32 at that rate; the library is compiled without packed FP32);
                beside it the same launch's LDS read rate (LDS instructions per
                launch from the committed rocprofv3 counter summary, each a
                16-byte read by 64 lanes) against the LDS peak (256 B/clk/CU x
                256 CUs x 2.4 GHz = 157.3 TB/s) and its HBM traffic (counter
                bytes per launch) against 8 TB/s; `bound` names the resource
                closest to its peak. Counter figures are used only when they
                were taken on the current kernel source, else null
  hbm           bytes of a step over the step time, against 8 TB/s, by two
                definitions: compulsory (each operator once, the input, the
                stage-1 result written and read back, the output; per
                direction) and io (operators once, inputs and outputs only)
  cpu_baseline  the FP64 oracle timed on the host on a bounded sample of the
                same workload and scaled to one pair: one core, and beside it
                ("parallel") one process per host core, split by column
  step_ms       mean, median and minimum of the timed steps (value =
                batch/mean)
  bf16_weights  the same pair with BF16-stored weights (FP32 values and
                accumulation): rate and relative L2 distance from the FP32-weight
                results (default run only)
  serving       p50/p99 latency and throughput of a mixed stream of forward
                and adjoint requests on 64^3/128^3/192^3 grids at 1000 req/s
                (5000 requests), FP32 and BF16 weights, with the device-bound
                capacity of each and the BF16/FP32 ratios of capacity and p99
                (default run only; --no-serving skips it)

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--weights f32|bf16|f16]
                    [--basis constant|linear] [--n-rho N] [--aperture cylinder|square]
                    [--batch B]

--basis linear, --n-rho N (a stage-2 radial grid of N values instead of the
radii) and --aperture square (the columns spaced along a square instead of
the cylinder) measure the same workload on the widened operators; --batch B
applies B volumes per call (value still counts pairs). Those runs report no
cpu_baseline and no traffic (the counters were taken on the default operators
at batch 1).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SRT fwd+adjoint pairs/s at 256^3, HBM GB/s % of peak; serving p50/p99 latency"
PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X FP32 vector: 256 CUs x 128 FMA/clk x 2 FLOP x 2.4 GHz
PEAK_HBM_GBPS = 8000.0
# LDS reads: 256 bytes per clock per CU on gfx950, 256 CUs at 2.4 GHz
PEAK_LDS_TBPS = 256 * 256 * 2.4e9 / 1e12
LDS_BYTES_PER_INST = 64 * 16  # the stage kernels' LDS instructions are ds_read_b128
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage_kernels_pact256.json")
# the stage kernels and the operator format they walk (layout, chunk cut)
# the kernels and the operator format they walk (plus the flags they are built with)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2402_15641_amd", "csrc", f)
                  for f in ("apply.hip", "srt_internal.h", "tiled.hip", "plan.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    from paper_2402_15641_amd import build as srt_build
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    common = [f for f in srt_build.COMMON if not os.path.isabs(f)]  # not the include paths
    flags = [common, srt_build.DEVICE_FLAGS, sorted(srt_build.FILE_FLAGS.items())]
    h.update(json.dumps(flags).encode())
    return h.hexdigest()


def counter_record(kernel: str):
    """Per-launch counter figures of `kernel` from the committed summary, if
    they were taken on the current kernel source (else None)."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec.get("kernels", {}).get(kernel)


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` (calibrated FETCH_SIZE + WRITE_SIZE)."""
    k = counter_record(kernel)
    return None if not k else k["fetch_bytes"] + k["write_bytes"]


def measured_lds_bytes(kernel: str):
    """LDS bytes read per launch of `kernel` (SQ_INSTS_LDS x 1 KiB)."""
    k = counter_record(kernel)
    return None if not k or "sq_insts_lds" not in k else k["sq_insts_lds"] * LDS_BYTES_PER_INST


def _oracle_sample(ap, F64, cols, heights, barrier=None):
    """Assembles the sample's operators, then times the oracle's forward and
    adjoint transforms (CRT12 and CRT34 and their transposes) of the columns
    `cols` with CRT34 on `heights`: (CRT12 s, CRT34 s, assembly s)."""
    from oracle import geometry as geo, srt as osrt
    t0 = time.perf_counter()
    a34 = geo.assemble_a34(ap, heights=heights)
    a12s = [geo.assemble_a12(ap, ap.angles[a]) for a in cols]
    t_asm = time.perf_counter() - t0
    if barrier is not None:
        barrier.wait()  # every process applies at the same time
    t1 = t2 = 0.0
    for A in a12s:
        s = time.perf_counter()
        G = osrt.crt12(A, F64)
        t1 += time.perf_counter() - s
        s = time.perf_counter()
        Y = osrt.crt34(a34, G, ap.n_z, ap.n_radii)
        Gp = osrt.crt34_t(a34, Y, ap.mz)
        t2 += time.perf_counter() - s
        s = time.perf_counter()
        osrt.crt12_t(A, Gp, ap.ms)
        t1 += time.perf_counter() - s
    return t1, t2, t_asm


def _oracle_worker(ap, F64, cols, heights, barrier, queue):
    queue.put(_oracle_sample(ap, F64, cols, heights, barrier))


def cpu_baseline(ap, F64, n_cols=32, h_stride=8, max_procs=16):
    """The oracle (FP64, scipy CSR) on a bounded sample: forward and adjoint
    for n_cols evenly spaced columns, with the stage-2 operator restricted to
    every h_stride-th sensor height; stage-1 time is scaled by the columns
    left out, stage-2 time also by the heights left out. Timed once on one
    core, then with one process per host core (at most max_procs), the
    columns split between them and applied concurrently. Runs before the GPU
    is touched, so the worker processes are plain forks of a CPU-only
    process."""
    import multiprocessing as mp
    import platform
    cols = np.linspace(0, ap.n_angles, n_cols, endpoint=False).astype(int)
    heights = list(range(0, ap.n_z, h_stride))
    scale = ap.n_angles / n_cols
    t1, t2, t_asm = _oracle_sample(ap, F64, cols, heights)
    t_pair = t1 * scale + t2 * scale * h_stride
    procs = max(1, min(max_procs, len(os.sched_getaffinity(0)), n_cols))
    ctx = mp.get_context("fork")
    barrier, queue = ctx.Barrier(procs), ctx.Queue()
    parts = np.array_split(cols, procs)
    workers = [ctx.Process(target=_oracle_worker, args=(ap, F64, part, heights, barrier, queue))
               for part in parts]
    for w in workers:
        w.start()
    res = [queue.get() for _ in workers]
    for w in workers:
        w.join()
    wall = max(a + b * h_stride for a, b, _ in res)  # concurrent: the slowest process
    t_pair_par = wall * scale
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads_env = {k: os.environ[k] for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                               "MKL_NUM_THREADS") if k in os.environ}
    return {"value": 1.0 / t_pair, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_cols} of {ap.n_angles} columns, stage 2 on {len(heights)} of "
                      f"{ap.n_z} heights, forward+adjoint, scaled to one full pair "
                      f"(sample apply {t1 + t2:.1f} s, assembly {t_asm:.1f} s not counted)",
            "seconds_per_pair": t_pair,
            "parallel": {"value": 1.0 / t_pair_par, "unit": "pairs/s", "cores": procs,
                         "kind": "oracle",
                         "sample": f"the same {n_cols} columns split over {procs} processes "
                                   "(one thread each) applied concurrently; slowest process, "
                                   "scaled like the one-core figure",
                         "seconds_per_pair": t_pair_par},
            "host": {"cpu": model, "affinity_cores": len(os.sched_getaffinity(0)),
                     "threads_env": threads_env}}


def serving_leg(rate=1000.0, requests=5000):
    """p50/p99 latency and throughput of the mixed serving stream at one
    arrival rate, FP32 and BF16 weights (the full rate sweep is
    paper_2402_15641_amd.serve_bench)."""
    from paper_2402_15641_amd.serve_bench import serving_mix
    t0 = time.perf_counter()
    recs = serving_mix([rate], seconds=requests / rate, min_requests=requests, pool=2)
    out = {"workload": "grids 64^3/128^3/192^3 drawn uniformly, N x N x 4N apertures, 70% "
                       "forward / 30% adjoint, Poisson arrivals, batches of up to 8 on 4 "
                       "streams, admission by device-memory footprint (16 GiB)",
           "rate_rps": rate}
    for r in recs:
        w = out.setdefault(r["weights"], {})
        if "device_bound_capacity_rps" in r:
            w["capacity_rps"] = r["device_bound_capacity_rps"]
        else:
            w.update({k: r[k] for k in ("p50_ms", "p99_ms", "mean_ms", "throughput_rps",
                                        "requests")})
    # BF16 against FP32 weights: by device-bound capacity (throughput at a
    # rate below capacity only follows the arrivals) and by p99 latency
    if "f32" in out and "bf16" in out:
        out["bf16_over_f32"] = {
            "capacity": out["bf16"]["capacity_rps"] / out["f32"]["capacity_rps"],
            "p99": out["bf16"]["p99_ms"] / out["f32"]["p99_ms"]}
    log(f"serving leg {time.perf_counter() - t0:.1f} s")
    return out


def main():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--weights", default="f32", choices=["f32", "bf16", "f16"])
    p.add_argument("--workload", default="pact256", choices=["pact256", "grid128"])
    p.add_argument("--basis", default="constant", choices=["constant", "linear"])
    p.add_argument("--n-rho", type=int, default=0,
                   help="stage-2 radial grid of this many values (0: the radii)")
    p.add_argument("--aperture", default="cylinder", choices=["cylinder", "square"],
                   help="square: the same columns spaced along a square of half-side R "
                        "(columns anywhere) instead of the cylinder")
    p.add_argument("--batch", type=int, default=1,
                   help="volumes per apply (the phantom repeated); value stays pairs/s")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-serving", action="store_true",
                   help="skip the serving leg (the mixed request stream at 1000 req/s)")
    p.add_argument("--profile-copy", action="store_true",
                   help="also run one 1 GiB read + 1 GiB write kernel (torch.neg; counter "
                        "calibration for FETCH_SIZE / WRITE_SIZE)")
    args = p.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "angle-sharded path is design only", file=sys.stderr)
        sys.exit(2)

    from srt_inputs import config, phantoms, square_columns, with_rho_grid

    if args.batch < 1:
        p.error("--batch must be at least 1")
    nb = args.batch
    variant = (args.basis != "constant" or args.n_rho > 0 or args.aperture != "cylinder"
               or nb != 1)
    ap = config(args.workload)
    t0 = time.perf_counter()
    F64 = phantoms.phantom(ap)
    if args.n_rho > 0:
        ap = with_rho_grid(ap, args.n_rho)
    if args.aperture == "square":
        ap = square_columns(ap, ap.radius)
    log(f"phantom {time.perf_counter() - t0:.1f} s")
    F_in = F64.astype(np.float32).astype(np.float64)  # the values the GPU receives
    cpu = None
    if not args.no_cpu_baseline and not variant:
        t0 = time.perf_counter()
        cpu = cpu_baseline(ap, F_in)
        log(f"cpu baseline {time.perf_counter() - t0:.1f} s: {cpu['value']:.4f} pairs/s on 1 core, "
            f"{cpu['parallel']['value']:.4f} on {cpu['parallel']['cores']}")

    import torch
    from paper_2402_15641_amd import SRTPlan, binding as B

    if not torch.cuda.is_available():
        log("bench.py needs a ROCm device")
        sys.exit(1)
    vol = torch.from_numpy(F64).float().cuda()
    if nb > 1:
        vol = vol.expand((nb,) + tuple(vol.shape)).contiguous()

    t0 = time.perf_counter()
    plan = SRTPlan.from_geometry(ap, value_dtype="f32", weight_dtype=args.weights,
                                 basis=args.basis)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    info = plan.info
    log(f"plan {t_plan:.2f} s {info}")
    lead = (nb,) if nb > 1 else ()
    ws = plan.workspace(nb)
    data = torch.empty(lead + tuple(ap.data_shape), device="cuda")
    back = torch.empty(lead + tuple(ap.vol_shape), device="cuda")
    stream = torch.cuda.current_stream()

    if args.profile_copy:
        src = torch.ones(1 << 28, device="cuda")  # 1 GiB of FP32
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)  # a kernel of its own name: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        plan.forward(vol, out=data, workspace=ws)
        plan.adjoint(data, out=back, workspace=ws)
    torch.cuda.synchronize()

    B.srt_plan_set_timing(plan.handle, True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    marks[0].record(stream)
    for i in range(args.steps):
        plan.forward(vol, out=data, workspace=ws)
        plan.adjoint(data, out=back, workspace=ws)
        marks[i + 1].record(stream)
    torch.cuda.synchronize()
    ms_per_step = marks[0].elapsed_time(marks[-1]) / args.steps
    steps_ms = [marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)]
    fwd_ms, n_f = B.srt_plan_stage_times(plan.handle, False)
    adj_ms, n_a = B.srt_plan_stage_times(plan.handle, True)
    B.srt_plan_set_timing(plan.handle, False)
    fwd_ms = [t / n_f for t in fwd_ms]
    adj_ms = [t / n_a for t in adj_ms]
    log("stage ms fwd", [round(t, 3) for t in fwd_ms], "adj", [round(t, 3) for t in adj_ms])

    # Algorithmic FLOPs per launch of each sparse stage (2 per multiply-add).
    nnz12, nnz34 = info["nnz_a12"], info["nnz_a34"]
    stages = {
        "stage1_fwd": (fwd_ms[1], 2.0 * nnz12 * ap.mz * nb),
        "stage2_fwd": (fwd_ms[3], 2.0 * nnz34 * ap.n_angles * nb),
        "stage2_adj": (adj_ms[1], 2.0 * nnz34 * ap.n_angles * nb),
        "stage1_adj": (adj_ms[3], 2.0 * nnz12 * ap.mz * nb),
    }
    dom = max(stages, key=lambda k: stages[k][0])
    dom_ms, dom_flop = stages[dom]
    achieved = dom_flop / (dom_ms * 1e-3) / 1e12
    counters_ok = not variant and args.weights == "f32"  # the summary's configuration
    traffic = measured_traffic(dom) if counters_ok else None
    lds_bytes = measured_lds_bytes(dom) if counters_ok else None
    # HBM bytes the counters saw per launch, over each stage kernel's time
    measured = {}
    if counters_ok:
        for k, (k_ms, _) in stages.items():
            b = measured_traffic(k)
            if b is not None:
                measured[k] = b / (k_ms * 1e-3) / 1e9
    frac_alu = achieved / PEAK_FP32_VALU_TFLOPS
    lds = None
    if lds_bytes is not None:
        lds_tbps = lds_bytes / (dom_ms * 1e-3) / 1e12
        lds = {"achieved": lds_tbps, "peak": PEAK_LDS_TBPS, "unit": "TB/s",
               "frac": lds_tbps / PEAK_LDS_TBPS, "bytes_per_launch": lds_bytes,
               "bytes_per_fma": lds_bytes / (dom_flop / 2)}
    fractions = {"alu": frac_alu}
    if lds:
        fractions["lds"] = lds["frac"]
    if traffic is not None:
        fractions["hbm"] = traffic / (dom_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS
    bound = max(fractions, key=fractions.get)

    wb = {"f32": 4, "bf16": 2, "f16": 2}[args.weights]
    op_bytes = 2 * (nnz12 + nnz34) * (4 + wb)  # operator and its transpose, once each
    vol_b = 4 * nb * int(np.prod(ap.vol_shape))
    dat_b = 4 * nb * int(np.prod(ap.data_shape))
    g_b = 4 * nb * ap.n_angles * info["live_radii"] * ap.mz  # stage-1 result (live rho cells)
    io_bytes = op_bytes + 2 * (vol_b + dat_b)
    comp_bytes = io_bytes + 2 * 2 * g_b  # plus G written and read back, each direction
    step_s = ms_per_step * 1e-3

    result = {
        "metric": METRIC,
        "value": 1000.0 * nb / ms_per_step,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.weights == "f32" else f"f32 (weights {args.weights})",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: " + ("256^3 voxels at 0.1 mm, R=15.36 mm, "
                                                        "512 columns x 256 heights x 1024 radii"
                                                        if args.workload == "pact256" else
                                                        "128^3 on [-1,1]^3, R=1.3, 128 x 128 x 512"),
                   "batch": nb, "weights": args.weights, "phantom": "seeded",
                   "basis": args.basis, "n_rho": info["n_rho"], "aperture": args.aperture,
                   "nnz_a12": nnz12, "nnz_a34": nnz34, "plan_build_s": round(t_plan, 3)},
        "roofline": {"bound": bound, "kernel": dom, "achieved": achieved,
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": frac_alu, "traffic": traffic,
                     "launch_ms": dom_ms, "flop_per_launch": dom_flop,
                     "fractions": fractions, "lds": lds},
        "hbm": {"compulsory_bytes_per_step": comp_bytes,
                "achieved_gbps": comp_bytes / step_s / 1e9, "peak_gbps": PEAK_HBM_GBPS,
                "frac": comp_bytes / step_s / 1e9 / PEAK_HBM_GBPS,
                "io_bytes_per_step": io_bytes, "io_gbps": io_bytes / step_s / 1e9,
                "io_frac": io_bytes / step_s / 1e9 / PEAK_HBM_GBPS,
                "measured_stage_gbps": measured or None},
        "step_ms": {"mean": ms_per_step, "median": float(np.median(steps_ms)),
                    "min": float(np.min(steps_ms))},
        "stage_ms": {"forward": fwd_ms, "adjoint": adj_ms},
        "cpu_baseline": cpu,
    }
    if not variant and args.weights == "f32":
        # the same pair with BF16-stored weights (FP32 values and accumulation)
        p16 = SRTPlan.from_geometry(ap, value_dtype="f32", weight_dtype="bf16")
        d16 = torch.empty_like(data)
        b16 = torch.empty_like(back)
        for _ in range(args.warmup):
            p16.forward(vol, out=d16, workspace=ws)
            p16.adjoint(d16, out=b16, workspace=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            p16.forward(vol, out=d16, workspace=ws)
            p16.adjoint(d16, out=b16, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms16 = e0.elapsed_time(e1) / args.steps
        result["bf16_weights"] = {
            "value": 1000.0 / ms16, "unit": "pairs/s", "ms_per_step": ms16,
            "rel_l2_forward_vs_f32_weights": float((d16 - data).norm() / data.norm()),
            "rel_l2_adjoint_vs_f32_weights": float((b16 - back).norm() / back.norm())}
        p16.close()
    plan.close()
    if not variant and not args.no_serving:
        result["serving"] = serving_leg()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
