"""Throughput of the iPiano-FoE despeckling hot path on one MI355X.

One step = one full solve of the 512x512 single-look workload (init, 300 iPiano
iterations with backtracking, output) on synthetic input resident in HBM.
Prints one JSON line:
  value      Mpixel-iterations/s = H*W*accepted_iterations / wall time per step
  roofline   the fused trial kernel against the FP32 peak (algorithmic flops per launch /
             its mean launch duration from per-launch HIP event pairs)
  cpu_baseline  the FP64 oracle on the host cores over a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Mpixel-iters/s iPiano-FoE on 1 GPU; time-to-PSNR vs plain FP32; roofline %"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 (vector and matrix)
NF, KK = 48, 49
FLOP_PER_PX_TRIAL = 2 * 2 * NF * KK   # forward bank on x+ and adjoint bank, one FMA = 2 flop


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(pr, bank, theta, seconds_target=15.0):
    import oracle
    p = oracle.Params(lam1=pr.lam1, lam2=pr.lam2)
    H, W = pr.f.shape
    # calibrate on 2 iterations, then run a bounded sample
    t = time.perf_counter()
    r = oracle.ipiano(p, pr.f, bank, theta, 2, L0=1.0)
    t2 = time.perf_counter() - t
    iters = int(max(2, min(60, seconds_target / max(t2 / 2, 1e-3))))
    t = time.perf_counter()
    r = oracle.ipiano(p, pr.f, bank, theta, iters, L0=1.0)
    dt = time.perf_counter() - t
    n_acc = int(r.stats.shape[0])
    return {"value": H * W * n_acc / dt / 1e6, "unit": "Mpixel-iters/s", "cores": oracle.get_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle, same 512x512 input, first {n_acc} iterations from x0 = log f "
                      f"({int(r.stats[:, 4].sum())} trials), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the workload is a single-GPU solve; multi-GPU runs are not "
              "part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1404_5344_amd as foe
    import synth

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    pr = synth.config2()
    bank, theta = synth.dct_bank(), synth.theta_weights(2)
    H, W = pr.f.shape
    p = foe.default_params(H, W, lambda1=pr.lam1, lambda2=pr.lam2, max_iters=args.iters, looks=1)
    stream = torch.cuda.current_stream()
    s = foe.Solver(p, bank, theta, stream=stream)
    f = torch.from_numpy(pr.f).to(dev)
    out = torch.empty_like(f)
    log(f"bench: {H}x{W}, {args.iters} iterations, warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        s.solve(f, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters_total = 0
    trials_total = 0
    for k in range(args.steps):
        r = s.solve(f, out=out)
        iters_total += r.summary["iters_done"]
        trials_total += r.summary["total_trials"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    psnr = synth.psnr(out.cpu().numpy(), pr.clean)
    log(f"bench: {dt * 1e3 / args.steps:.3f} ms/step, psnr {psnr:.4f} dB, trials/iter {trials_total / iters_total:.4f}")

    # dominant kernel: fused trial kernel, mean of per-launch HIP event pairs on the solver stream
    ms_launch = s.profile_trial(50)
    flop = FLOP_PER_PX_TRIAL * H * W
    achieved = flop / (ms_launch * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                "kernel": "fused_valu_kernel", "ms_per_launch": round(ms_launch, 5),
                "flop_per_launch": flop}
    value = H * W * iters_total / dt / 1e6
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpixel-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512x512 shapes+cosine image, L=1 speckle, COMBINED model (lambda 160, 0.004), "
                               "48 DCT 7x7 filters, SYMMETRIC boundary, beta 0.8, backtracking, "
                               f"{args.iters} iterations per step",
                   "pixels": H * W, "iterations": args.iters, "trials_per_iter": round(trials_total / iters_total, 4),
                   "psnr_db": round(psnr, 4)},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        res["cpu_baseline"] = cpu_baseline(pr, bank, theta)
    s.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
