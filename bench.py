"""Benchmark: candidate reductions scored per second on the 1000-node,
24-snapshot feeder (whole search per step: planning, load flow, every
segment's 2^k candidates, arg-min, state update, Y_Kron and final errors).

Prints ONE JSON line.  `value` = candidates scored per second with the inputs
resident in HBM.  `roofline` describes the dominant kernel (the FP64 scoring
kernel) from HIP-event timings taken in the timed region; `cpu_baseline` is
the FP64 CPU oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (256 CUs x 2.4 GHz x 128 flop/clk)
FP32_VECTOR_PEAK_TFLOPS = 157.3


def cpu_baseline(f, seconds=12.0):
    """FP64 oracle scoring masks of the first segment (initial state), as many
    as fit in about `seconds` of one host core."""
    import numpy as np
    import oracle
    V, I, st, _ = oracle.powerflow(f)
    keep = np.ones(f["n"], np.uint8)
    k = int((f["segment"] == 0).sum())
    done, t0, m0 = 0, time.perf_counter(), 0
    batch = 64
    while time.perf_counter() - t0 < seconds and m0 < (1 << k):
        masks = np.arange(m0, min(m0 + batch, 1 << k), dtype=np.uint32)
        oracle.score_masks(f, V, I, keep, 0, masks)
        done += len(masks)
        m0 += batch
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="candidates/s", cores=1, kind="oracle",
                sample=f"first {done} masks of segment 0 (k={k}) of the 1000-node 24-snapshot feeder, "
                       f"FP64 Kron elimination + reduced-network solve + scoring per mask, {dt:.1f} s on 1 core")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this search runs on one GPU; --gpus above 1 is not supported "
                                   "(see DESIGN.md for how segments would shard)"}))
        sys.exit(2)

    import torch
    from paper_2510_19608_amd import Reducer
    from synth_feeders import make_feeder

    f = make_feeder("c2", args.seed)
    R = Reducer(f, device="cuda:0", precision=args.precision, timing=True)
    ncand = int(R.sizes.n_candidates)
    for _ in range(args.warmup):
        R.run()
    torch.cuda.synchronize()
    kern_ms, flops = 0.0, 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        R.run()
        r = R.res
        kern_ms += r.score_kernel_ms
        flops += r.algorithmic_flops
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = R.result()
    ms_per_step = dt * 1e3 / args.steps
    launches = out["n_score_launches"] * args.steps
    achieved = flops / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else None
    line = {
        "metric": "candidate reductions scored/sec (1000-node, 24 snaps); time-to-optimal vs plain",
        "value": ncand * args.steps / dt,
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "c2: 1000-node synthetic three-phase feeder, 24 snapshots, "
                               "segments of 16 eligible nodes, exhaustive 2^16 masks per segment",
                   "seed": args.seed, "n_candidates": ncand, "segments": int(R.sizes.n_segments),
                   "precision": args.precision, "e_bar": f["e_bar"], "n_kept": int(out["n_kept"]),
                   "max_err": out["max_err"], "time_to_optimal_ms": ms_per_step,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": (achieved / FP64_VECTOR_PEAK_TFLOPS) if achieved else None,
                     "traffic": None, "kernel": "okr::k_score_fp64",
                     "avg_launch_us": kern_ms * 1e3 / max(launches, 1),
                     "flops_per_launch": flops / max(launches, 1)},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(f)
    R.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
