#!/usr/bin/env python3
"""Benchmark: morphed samples/s of the PDMP hot path on one MI355X.

One step = one pass of the hot path over one batch of the 2-D large workload
(1,048,576 prior samples, 64x64 hinges, l = 0.4, T = 50, eta = 0.02, 100 discs):
  Philox prior batch on the GPU -> collision labels before -> fused T-step Euler
  morph down grad c -> collision labels after.
The occupancy is fitted once per scene before the timed region.  Inputs are
resident in HBM when timing starts.

Prints one JSON line (metric, value, roofline of the dominant kernel, and the FP64
oracle timed on the host cores as `cpu_baseline`).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and the chip's unit counts (256 CUs, 2.4 GHz).
PEAK_FP32_VALU = 157.3e12          # FLOP/s, dense FP32 vector (packed issue)
# v_exp_f32 runs at half rate (8 cycles per wave64 on a 16-lane SIMD): 4 SIMDs x
# 16 lanes x 1/2 per clock per CU.  Measured on the part, it overlaps with
# independent VALU work, so the pair bound is max(flop time, exp time).
PEAK_EXP = 256 * 4 * 16 * 0.5 * 2.4e9
FLOPS_PER_PAIR = {2: 12, 3: 17}    # 5*dim + 2 algorithmic FP32 flops per sample-hinge pair


def alu_peak_tflops(dim):
    """Bound for one pair = f flops + 1 exp (max model), as FP32 TFLOP/s."""
    f = FLOPS_PER_PAIR[dim]
    t_pair = max(f / PEAK_FP32_VALU, 1.0 / PEAK_EXP)
    return f / t_pair / 1e12


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=1 << 17,
                   help="samples of the batch the oracle morphs for the CPU baseline")
    return p.parse_args()


def cpu_baseline(occ_np, x0_np, cfg, n_sample):
    import numpy as np
    import oracle as O
    idx = np.linspace(0, x0_np.shape[1] - 1, n_sample).astype(np.int64)
    xs = np.ascontiguousarray(x0_np[:, idx])
    t0 = time.perf_counter()
    O.morph_ws(occ_np, xs, cfg.T, cfg.eta)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "samples/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{n_sample} of the {x0_np.shape[1]} prior samples (evenly strided), "
                      f"full T={cfg.T} FP64 morph over all {occ_np.M} hinges; "
                      f"{dt:.2f} s wall"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2108_11775_amd as P
    from paper_2108_11775_amd import configs as K, inputs as I

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    cfg = K.C2
    dev = torch.device("cuda", 0)
    print(f"[bench] workload {cfg.name}: N={cfg.n_samples} T={cfg.T} M={cfg.n_hinges}", file=sys.stderr,
          flush=True)

    h = I.hinge_grid(2, cfg.grid, cfg.lo, cfg.hi)
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    wb = np.load(os.path.join(ROOT, "tests", "golden", "ws2d_1M.npy")).astype(np.float32)
    h_d = torch.from_numpy(h).to(dev)
    w_d = torch.from_numpy(wb).to(dev)
    dc_d, dr_d = torch.from_numpy(dc).to(dev), torch.from_numpy(dr).to(dev)
    occ = P.Occupancy(h_d, w_d, cfg.lengthscale)

    N = cfg.n_samples
    seed = I.philox_seed(cfg.cfg_id)
    x0 = torch.empty((2, N), dtype=torch.float32, device=dev)
    x1 = torch.empty_like(x0)
    lab0 = torch.empty(N, dtype=torch.uint8, device=dev)
    lab1 = torch.empty_like(lab0)
    hit0 = torch.zeros(1, dtype=torch.int64, device=dev)
    hit1 = torch.zeros(1, dtype=torch.int64, device=dev)
    lo, hi = [cfg.lo] * 2, [cfg.hi] * 2

    ev = []  # (start, end) around each morph launch in the timed region

    def step(i, record):
        P.uniform_samples(seed, i, lo, hi, N, out=x0)
        P.label_points_discs(dc_d, dr_d, x0, count=True, out=lab0, hit=hit0)
        if record:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
        P.morph_samples(occ, x0, cfg.T, cfg.eta, out=x1)
        if record:
            e1.record()
            ev.append((e0, e1))
        P.label_points_discs(dc_d, dr_d, x1, count=True, out=lab1, hit=hit1)

    for i in range(args.warmup):
        step(1000 + i, False)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_start.record()
    for i in range(args.steps):
        step(i, True)
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    morph_ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
    free_before = 1.0 - hit0.item() / N
    free_after = 1.0 - hit1.item() / N
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step, morph {morph_ms:.3f} ms",
          file=sys.stderr, flush=True)

    pairs = N * cfg.T * cfg.n_hinges
    achieved = pairs * FLOPS_PER_PAIR[2] / (morph_ms * 1e-3) / 1e12
    peak = alu_peak_tflops(2)
    out = {
        "metric": "morphed samples/s (T steps) + collision-free fraction; amortised vs plain morph",
        "value": N / (ms_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded disc world, Philox prior samples)",
        "config": {"workload": "plain morph 2-D large: 1,048,576 samples, 64x64 hinges, "
                               "l=0.4, T=50, eta=0.02, 100 discs",
                   "N": N, "T": cfg.T, "M": cfg.n_hinges, "eta": cfg.eta,
                   "weights": "oracle-fitted (tests/golden/ws2d_1M.npy)"},
        "collision_free_before": free_before,
        "collision_free_after": free_after,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "k_rbf<2,2,1,1024,kMorph>",
                     "kernel_ms": morph_ms},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        x0_np = np.empty((2, N), np.float32)
        P.uniform_samples(seed, 0, lo, hi, N, out=x0)
        x0_np[:] = x0.cpu().numpy()
        occ_np = O.Occupancy(h, wb[:-1], float(wb[-1]), cfg.lengthscale)
        print("[bench] cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(occ_np, x0_np, cfg, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
