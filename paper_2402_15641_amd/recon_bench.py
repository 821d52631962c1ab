"""Reconstruction benchmark: iterations per second at PACT scale.

Workload: the 256^3 grid at 0.1 mm with 512 columns x 256 heights x 1024
radii (FP32), data g = SRT of the 200-cylinder phantom plus 1% Gaussian
noise, starting from zero. One iteration is one forward, one adjoint and the
vector updates, all on the device: srt_cgls (least squares) or srt_nnls
(least squares with f >= 0, step 1/(1.05 x the srt_opnorm2 estimate after
30 power steps, timed separately)). Prints one JSON line with the iteration
rate and the residual or misfit history. A call is timed at the requested
number of iterations and at one iteration: ms_total is the first,
ms_per_iter the difference per further iteration (what an iteration costs
once the solver runs; CGLS also starts with r = g - A f0 and s = A^T r).

    python -m paper_2402_15641_amd.recon_bench [--iters 10] [--weights f32|bf16]
                                               [--method cgls|nnls]
"""
from __future__ import annotations

import argparse
import json
import os
import sys


def main():
    ap_ = argparse.ArgumentParser()
    ap_.add_argument("--iters", type=int, default=10)
    ap_.add_argument("--weights", default="f32", choices=["f32", "bf16", "f16"])
    ap_.add_argument("--method", default="cgls", choices=["cgls", "nnls"])
    args = ap_.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import torch
    from srt_inputs import config, phantoms
    from paper_2402_15641_amd import SRTPlan, binding as B

    ap = config("pact256")
    plan = SRTPlan.from_geometry(ap, value_dtype="f32", weight_dtype=args.weights)
    F = torch.from_numpy(phantoms.phantom(ap)).float().cuda()
    g = plan.forward(F)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    g += 0.01 * g.abs().max() * torch.randn(g.shape, device="cuda", generator=gen)
    if args.method == "nnls":
        return bench_nnls(plan, F, g, args)
    ws = torch.empty(B.srt_cgls_workspace(plan.handle, 1, args.iters), dtype=torch.uint8,
                     device="cuda")
    plan.cgls(g, 2, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    ms1 = timed(lambda: plan.cgls(g, 1, workspace=ws, want_resid=False))[0]
    ms, (f, _) = timed(lambda: plan.cgls(g, args.iters, workspace=ws, want_resid=False))
    _, resid = plan.cgls(g, args.iters, workspace=ws)
    err = float((f - F).norm() / F.norm())
    per = (ms - ms1) / (args.iters - 1) if args.iters > 1 else ms
    print(json.dumps({"workload": "pact256 CGLS", "weights": args.weights, "iters": args.iters,
                      "ms_total": ms, "ms_one_iter_call": ms1, "ms_per_iter": per,
                      "iters_per_s": 1000.0 / per,
                      "normal_residual": [float(x) for x in resid[:, 0]],
                      "rel_error_vs_phantom": err}), flush=True)
    plan.close()


def timed(fn):
    """Milliseconds of one call on the current stream (events around it), and
    its result."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), out


def bench_nnls(plan, F, g, args):
    import time
    import torch
    from paper_2402_15641_amd import binding as B
    t0 = time.perf_counter()
    L = plan.opnorm2(30)
    t_norm = time.perf_counter() - t0
    step = 1.0 / (1.05 * L)
    ws = torch.empty(B.srt_nnls_workspace(plan.handle, 1, args.iters), dtype=torch.uint8,
                     device="cuda")
    plan.nnls(g, 2, step=step, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    ms1 = timed(lambda: plan.nnls(g, 1, step=step, workspace=ws, want_resid=False))[0]
    ms, (f, _, _) = timed(lambda: plan.nnls(g, args.iters, step=step, workspace=ws,
                                            want_resid=False))
    _, resid, _ = plan.nnls(g, args.iters, step=step, workspace=ws)
    err = float((f - F).norm() / F.norm())
    per = (ms - ms1) / (args.iters - 1) if args.iters > 1 else ms
    print(json.dumps({"workload": "pact256 NNLS (FISTA)", "weights": args.weights,
                      "iters": args.iters, "opnorm2": L, "opnorm2_s": t_norm, "step": step,
                      "ms_total": ms, "ms_one_iter_call": ms1, "ms_per_iter": per,
                      "iters_per_s": 1000.0 / per,
                      "misfit": [float(x) for x in resid[:, 0]],
                      "min_value": float(f.min()), "rel_error_vs_phantom": err}), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
