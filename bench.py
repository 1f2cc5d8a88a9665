#!/usr/bin/env python3
"""Benchmark: morphed samples/s of the PDMP hot path on one MI355X.

Headline step (timed K times) = one pass of the hot path over one batch of the 2-D
large workload (1,048,576 prior samples, 64x64 hinges, l = 0.4, T = 50,
eta = 0.02, 100 discs):
  Philox prior batch on the GPU -> collision labels before -> fused T-step Euler
  morph down grad c (spatially ordered: counting sort, then the grid kernel that
  skips exact zeros) -> collision labels after.
The occupancy is fitted on the GPU once per scene, before the timed region (200
gradient-descent steps on 10^4 labelled points).  Inputs are resident in HBM when
timing starts.

The other workloads run once each after the headline and are reported under
"workloads": the small 2-D morph, the 7-DOF arm morph, the 3-D occupancy fit
(500 Adam steps on 2^20 points) and the amortised morph (residual MLP trained on
plain-morph pairs, plain-morph fallback) against the plain arm morph.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (256 CUs, 2.4 GHz).
PEAK_FP32_VALU = 157.3e12          # FLOP/s, dense FP32 vector
PEAK_FP32_MFMA = 157.3e12          # FLOP/s, dense FP32 matrix
PEAK_BF16_MFMA = 2.5e15            # FLOP/s, dense BF16 matrix
PEAK_F16_MFMA = 2.5e15             # FLOP/s, dense FP16 matrix
SIMDS, CLOCK_HZ = 1024, 2.4e9      # the peaks' SIMD count and clock
FLOPS_PER_PAIR = {2: 12, 3: 17}    # 5*dim + 2 algorithmic FP32 flops per sample-hinge pair


# HBM traffic per call of the headline's ordered morph (the counting sort's four kernels
# and k_grid2d_sorted) from the two rocprofv3 --pmc runs in
# profiles/k_grid2d_sorted_morph_ws2d_1M.md (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, the
# factors a plain 256 MiB device copy reads under the same counters).  Valid only
# while the kernels' sources (grid2d.hip and the headers it includes) are the ones
# the counters were taken on.
GRID2D_SOURCES = ("grid2d.hip", "grid2d_stage.h", "mfma_split.h", "pdmp_common.h")
GRID2D_TRAFFIC = {"bytes": (14740.7 * 2.0 + 21232.5) * 1024,
                  "sha256": "e1644aa66723385458e31679a26853df0792cb9f60c72e43dac63eaf38b74bca"}


def grid2d_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in GRID2D_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_11775_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def grid2d_traffic():
    return GRID2D_TRAFFIC["bytes"] if grid2d_sources_sha() == GRID2D_TRAFFIC["sha256"] else None


# Instructions per wave-step (32 samples, one Euler step) of the ordered kernel from one
# rocprofv3 --pmc run on the same call (SQ_INSTS_* over 2^20 / 32 x 50 wave-steps,
# profiles/k_grid2d_sorted_morph_ws2d_1M.md), beside the unordered kernel's on the same
# batch: the MFMAs the exact-zero skipping leaves and the VALU work it keeps.  Reported
# only while the sources are the ones the counters were taken on.
GRID2D_COUNTS = {"valu": 395.3, "mfma": 19.23, "salu": 92.8, "lds": 22.3,
                 "unordered_valu": 581.0, "unordered_mfma": 48.0,
                 "sha256": GRID2D_TRAFFIC["sha256"]}


def grid2d_counts():
    u = GRID2D_COUNTS
    if grid2d_sources_sha() != u["sha256"]:
        return None
    return {"unit": "instructions per wave-step", "valu": u["valu"], "mfma": u["mfma"],
            "salu": u["salu"], "lds": u["lds"],
            "unordered_kernel": {"valu": u["unordered_valu"], "mfma": u["unordered_mfma"]},
            "mfma_executed_fraction": u["mfma"] / u["unordered_mfma"],
            "source": "profiles/k_grid2d_sorted_morph_ws2d_1M.md"}


# Issue costs measured on this device at the start of the run (pdmp_issue_rates:
# shader-clock cycles per wave64 instruction on one SIMD); filled in by main().
RATES = {}


def alu_peak_tflops(dim):
    """The pairwise kernels' ALU ceiling for their own work, 5 dim + 2 FP32 flops and
    one exponential per pair, at the published 157.3 TF for the flops and the measured
    v_exp_f32 cost for the exponential (the mixed probe shows the two classes adding on
    the issue port, not overlapping), at the peaks' 2.4 GHz."""
    f = FLOPS_PER_PAIR[dim]
    exp_per_s = SIMDS * 64 * CLOCK_HZ / RATES["v_exp_f32"]
    return f / (f / PEAK_FP32_VALU + 1.0 / exp_per_s) / 1e12


def grid_ceiling(kind, n_units, per_unit):
    """Achievable time of a grid kernel under its own formulation, from the measured
    issue costs: per wave-step (2-D: one wave of 32 samples through one step; arm: one
    wave of 4 configurations x 8 body points through one link) the MFMA pipe's time for
    the split products and the least VALU time the formulation needs (the exponentials,
    offsets, splits of the B operands and the contractions on the accumulator layout;
    kernel overhead not counted).  Perfect overlap of the two gives the ceiling; the
    sum is the time with none.  At the peaks' 2.4 GHz."""
    c_f, c_e = RATES["v_fma_f32"], RATES["v_exp_f32"]
    c_c, c_m = RATES["v_cvt_pk_f16_f32"], RATES["v_fma_mix_f32"]
    x_val = 3 * c_f + c_e + 2 * (c_c + c_m)     # offset, argument, exp, ex dx, 2 FP16 splits
    if kind == "ws2d":
        xv, yr = per_unit["x_per_lane"], per_unit["y_per_lane"]
        valu = xv * x_val + yr * (6 * c_f + c_e)    # y row: offset, argument, exp, 3 FMA + 1 mul
    else:
        xv, yv, zv, fm = (per_unit[k] for k in ("x_per_lane", "y_per_lane", "z_per_lane",
                                                "contraction_fma_per_lane"))
        valu = xv * x_val + (yv + zv) * (3 * c_f + c_e) + fm * c_f
    mfma = per_unit["mfma"] * RATES["v_mfma_f32_32x32x16_f16"]
    per_simd = n_units / SIMDS
    to_ms = per_simd / CLOCK_HZ * 1e3
    return {"formulation": "dense: every hinge block and row tile of the factorised sums",
            "valu_cycles_per_unit": valu, "mfma_cycles_per_unit": mfma,
            "ceiling_ms": max(valu, mfma) * to_ms, "no_overlap_ms": (valu + mfma) * to_ms,
            "unit": per_unit["unit"], "units": n_units}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--settle-s", type=float, default=0.5,
                   help="seconds of untimed headline steps before the warm-up steps, so that "
                        "the GPU clocks have left their idle state")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=1 << 17,
                   help="prior samples the FP64 oracle morphs for the CPU baseline")
    p.add_argument("--headline-only", action="store_true",
                   help="skip the secondary workloads (profiling runs)")
    p.add_argument("--dense", action="store_true",
                   help="headline with the pairwise kernel instead of the grid factorisation")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a plain 256 MiB device copy first (scales profiler byte counters)")
    p.add_argument("--workloads", default="all",
                   help="comma-separated secondary workloads after the headline: small, "
                        "density, culled, pipeline, tanh, arm (the 3-D fit and the arm "
                        "morph), amortised; or all")
    p.add_argument("--rrt-runs", type=int, default=0,
                   help="runs of the plane-RRT time-to-solution comparison (morph sampler "
                        "against the prior) in the pipeline workload; 0 skips it")
    p.add_argument("--no-trajectory-check", action="store_true",
                   help="skip the oracle's one-step check along the bench's own GPU paths "
                        "(it runs with the CPU baseline)")
    p.add_argument("--train-epochs", type=int, default=None)
    p.add_argument("--train-batches", type=int, default=None)
    p.add_argument("--amortised-variants", action="store_true",
                   help="also train the amortised network's variants (samples whose output "
                        "lands occupied weighted up; a longer schedule with restarts) and "
                        "report each one's fallback-vs-collision-free frontier")
    return p.parse_args()


def median_ms(torch, f, reps=5):
    """Median over reps calls of f, each between its own pair of HIP events."""
    ts = []
    for _ in range(reps):
        t = Timer(torch)
        with t:
            f()
        ts.append(t)
    ms = sorted(t.ms() for t in ts)
    return ms[len(ms) // 2]


class Timer:
    """HIP events on torch's current stream (the stream every call is launched on)."""

    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()

    def ms(self):
        self.torch.cuda.synchronize()
        return self.a.elapsed_time(self.b)


def ws_scene(P, I, K, torch, cfg, dev, grid=True):
    """2-D disc world of a config with its occupancy fitted on the GPU."""
    h = I.hinge_grid(2, cfg.grid, cfg.lo, cfg.hi)
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    pts = I.uniform_points(cfg.cfg_id, K.STREAM_FIT, 2, cfg.fit_points, cfg.lo, cfg.hi)
    h_d = torch.from_numpy(h).to(dev)
    dc_d, dr_d = torch.from_numpy(dc).to(dev), torch.from_numpy(dr).to(dev)
    pts_d = torch.from_numpy(pts).to(dev)
    y = P.label_points_discs(dc_d, dr_d, pts_d)
    w = torch.zeros(h.shape[1] + 1, dtype=torch.float32, device=dev)
    t = Timer(torch)
    with t:
        loss = P.fit_occupancy(h_d, cfg.lengthscale, w, pts_d, y, cfg.fit_steps, cfg.fit_lr,
                               cfg.fit_l2, "gd", lr_bias=cfg.fit_lr_bias,
                               grid=(cfg.grid, cfg.grid) if grid else None)
    fit_ms = t.ms()
    occ = P.Occupancy(h_d, w, cfg.lengthscale, grid=(cfg.grid, cfg.grid) if grid else None)
    return dict(h=h, occ=occ, discs=(dc_d, dr_d), fit_ms=fit_ms,
                fit_loss=(float(loss[0]), float(loss[-1])), w=w)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(O, h, w, ell, x0_np, cfg, n_sample):
    """The FP64 oracle's morph on a strided sample of the headline batch, on all the
    host's threads and (on a sixteenth of that sample) on one."""
    import numpy as np
    idx = np.linspace(0, x0_np.shape[1] - 1, n_sample).astype(np.int64)
    xs = np.ascontiguousarray(x0_np[:, idx])
    wb = w.cpu().numpy()
    occ_np = O.Occupancy(h, wb[:-1], float(wb[-1]), ell)
    nt = O.num_threads()
    t0 = time.perf_counter()
    O.morph_ws(occ_np, xs, cfg.T, cfg.eta)
    dt = time.perf_counter() - t0
    n1 = max(1, n_sample // 16)
    O.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.morph_ws(occ_np, np.ascontiguousarray(xs[:, :n1]), cfg.T, cfg.eta)
        dt1 = time.perf_counter() - t0
    finally:
        O.set_num_threads(nt)
    return {"value": n_sample / dt, "unit": "samples/s", "cores": nt,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{n_sample} of the {x0_np.shape[1]} prior samples of one batch (evenly "
                      f"strided), full T={cfg.T} FP64 morph over all {h.shape[1]} hinges; "
                      f"{dt:.2f} s wall",
            "one_thread": {"value": n1 / dt1, "unit": "samples/s", "cores": 1,
                           "sample": f"the first {n1} of those samples; {dt1:.2f} s wall"}}


def trajectory_check(O, P, I, K, torch, hl, world):
    """The oracle's one-step check along the GPU's own paths on this run's GPU-fitted
    weights (the parity tests use oracle-fitted ones): the recording morph writes every
    state of a strided subset of the headline batch (and of the arm batch), the oracle
    takes one FP64 step from each recorded state, and the result is held to the
    one-step tolerance 1e-5 (|x'| + eta G_abs).  Beside it: the step Jacobian's figures
    at the visited states and the share of final states within the unscaled 1e-5 of
    the oracle's own T-step path."""
    import numpy as np
    res = {}
    cfg, occ = hl["cfg"], hl["sc"]["occ"]
    h = hl["sc"]["h"]
    wb = occ.weights.cpu().numpy()
    oo = O.Occupancy(h, wb[:-1], float(wb[-1]), cfg.lengthscale)
    x0 = P.uniform_samples(hl["seed"], 0, [cfg.lo] * 2, [cfg.hi] * 2, hl["N"])
    stride = 2048
    _, tr = P.morph_trajectory(occ, x0, cfg.T, cfg.eta, stride=stride)
    tr = tr.cpu().numpy()
    X = np.ascontiguousarray(tr[:-1].transpose(1, 0, 2).reshape(2, -1)).astype(np.float64)
    Y = tr[1:].transpose(1, 0, 2).reshape(2, -1)
    ref = O.morph_ws(oo, X, 1, cfg.eta)
    _, _, _, gabs = O.occ_grad(oo, X)
    err = np.abs(Y - ref)
    tol = 1e-5 * (np.abs(ref) + cfg.eta * gabs[None, :])
    _, _, mdet, meh = O.morph_ws(oo, X, 1, cfg.eta, diag=True)
    refT = O.morph_ws(oo, tr[0].astype(np.float64), cfg.T, cfg.eta)
    errT = np.abs(tr[-1] - refT).max(axis=0)
    res["ws2d_large"] = {
        "samples": int(tr.shape[2]), "stride": stride, "states": int(X.shape[1]),
        "one_step_max_err_over_tol": float((err / tol).max()),
        "one_step_within_tol": bool(np.all(err <= tol)),
        "share_final_within_unscaled_1e-5": float(
            np.mean(errT <= 1e-5 * np.maximum(1.0, np.abs(refT).max(axis=0)))),
        "max_eta_hess": float(meh.max()), "steps_det_nonpositive": int((mdet <= 0).sum())}
    if world is not None:
        c3 = K.C3
        arm, aocc = world["arm"], world["occ"]
        awb = aocc.weights.cpu().numpy()
        aoo = O.Occupancy(aocc.hinges.cpu().numpy(), awb[:-1], float(awb[-1]), c3.lengthscale)
        aarm = O.Arm(*I.dh_params(c3.cfg_id, c3.n_dof, c3.link_min, c3.link_max, c3.alpha),
                     c3.pts_per_link)
        q0 = P.uniform_samples(I.philox_seed(c3.cfg_id), 0, [c3.q_lo] * 7, [c3.q_hi] * 7,
                               c3.n_samples)
        stride = 1024
        _, tq = P.morph_trajectory(aocc, q0, c3.T, c3.eta, stride=stride, arm=arm)
        tq = tq.cpu().numpy()
        Q = np.ascontiguousarray(tq[:-1].transpose(1, 0, 2).reshape(7, -1)).astype(np.float64)
        Yq = tq[1:].transpose(1, 0, 2).reshape(7, -1)
        refq = O.morph_arm(aarm, aoo, Q, 1, c3.eta)
        scale = O.arm_step_scale(aarm, aoo, Q)
        errq = np.abs(Yq - refq)
        tolq = 1e-5 * (np.abs(refq) + c3.eta * scale[None, :])
        sub = tq[:, :, ::4]
        Qs = np.ascontiguousarray(sub[:-1].transpose(1, 0, 2).reshape(7, -1)).astype(np.float64)
        _, _, mdq, mehq = O.morph_arm(aarm, aoo, Qs, 1, c3.eta, diag=True, with_eh=True)
        refT = O.morph_arm(aarm, aoo, tq[0].astype(np.float64), c3.T, c3.eta)
        errT = np.abs(tq[-1] - refT).max(axis=0)
        res["arm7"] = {
            "configs": int(tq.shape[2]), "stride": stride, "states": int(Q.shape[1]),
            "one_step_max_err_over_tol": float((errq / tolq).max()),
            "one_step_within_tol": bool(np.all(errq <= tolq)),
            "share_final_within_unscaled_1e-5": float(
                np.mean(errT <= 1e-5 * np.maximum(1.0, np.abs(refT).max(axis=0)))),
            "diag_configs": int(sub.shape[2]), "max_eta_hess": float(mehq.max()),
            "steps_det_nonpositive": int((mdq <= 0).sum()),
            "paths_with_a_folding_step": int((mdq.reshape(c3.T, -1) <= 0).any(axis=0).sum())}
    return res


def headline(args, P, I, K, torch, dev):
    cfg = K.C2
    log(f"headline {cfg.name}: N={cfg.n_samples} T={cfg.T} M={cfg.n_hinges}")
    sc = ws_scene(P, I, K, torch, cfg, dev, grid=not args.dense)
    occ, (dc_d, dr_d) = sc["occ"], sc["discs"]
    log(f"GPU fit: {sc['fit_ms']:.1f} ms, loss {sc['fit_loss'][0]:.4f} -> {sc['fit_loss'][1]:.4f}")
    N = cfg.n_samples
    seed = I.philox_seed(cfg.cfg_id)
    x0 = torch.empty((2, N), dtype=torch.float32, device=dev)
    x1 = torch.empty_like(x0)
    lab0 = torch.empty(N, dtype=torch.uint8, device=dev)
    lab1 = torch.empty_like(lab0)
    hit0 = torch.zeros(1, dtype=torch.int64, device=dev)
    hit1 = torch.zeros(1, dtype=torch.int64, device=dev)
    lo, hi = [cfg.lo] * 2, [cfg.hi] * 2
    ev, sev = [], []
    # the spatially ordered morph's workspace (None on the pairwise path), allocated
    # once before the timed region
    mws = P.morph_workspace(occ, N, cfg.T)

    def step(i, record):
        if record:
            s_ = Timer(torch)
            s_.__enter__()
        P.uniform_samples(seed, i, lo, hi, N, out=x0)
        P.label_points_discs(dc_d, dr_d, x0, count=True, out=lab0, hit=hit0)
        if record:
            e = Timer(torch)
            e.__enter__()
        P.morph_samples_ws(occ, x0, cfg.T, cfg.eta, out=x1, ws=mws)
        if record:
            e.__exit__()
            ev.append(e)
        P.label_points_discs(dc_d, dr_d, x1, count=True, out=lab1, hit=hit1)
        if record:
            s_.__exit__()
            sev.append(s_)

    # clocks: the GPU leaves its idle state over some hundred milliseconds of work, so
    # untimed steps run for args.settle_s before the warm-up steps (not counted as steps)
    t_settle = time.perf_counter()
    n_settle = 0
    while time.perf_counter() - t_settle < args.settle_s:
        step(2000 + n_settle % 16, False)
        torch.cuda.synchronize()
        n_settle += 1
    for i in range(args.warmup):
        step(1000 + i, False)
    torch.cuda.synchronize()
    log(f"clock settling: {n_settle} untimed steps in {args.settle_s:.2f} s; "
        f"warmup done ({args.warmup} steps)")
    tt = Timer(torch)
    with tt:
        for i in range(args.steps):
            step(i, True)
    total_ms = tt.ms()
    ms_step = total_ms / args.steps
    kms = sorted(e.ms() for e in ev)
    morph_ms = sum(kms) / len(kms)
    morph_median = kms[len(kms) // 2] if len(kms) % 2 else 0.5 * (kms[len(kms) // 2 - 1] +
                                                                    kms[len(kms) // 2])
    sms = sorted(e.ms() for e in sev)
    step_median = sms[len(sms) // 2] if len(sms) % 2 else 0.5 * (sms[len(sms) // 2 - 1] +
                                                                   sms[len(sms) // 2])
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step (median {step_median:.3f}), "
        f"morph {morph_ms:.3f} ms (median {morph_median:.3f})")
    res = dict(cfg=cfg, N=N, ms_step=ms_step, step_median=step_median, morph_ms=morph_ms,
               morph_median=morph_median,
               free_before=1.0 - hit0.item() / N, free_after=1.0 - hit1.item() / N, sc=sc,
               seed=seed, x0=x0)
    G0 = G1 = cfg.grid
    if occ.grid:
        # the scheme the library ran, and the algorithmic work of the factorised
        # evaluation per sample and step: two G1 x G0 matrix-vector products, 4 G0 G1
        # FP32 flops, run on the matrix cores at FP32 accuracy as split products
        scheme, nprod = P.split_scheme(occ)
        fp32_tf = N * cfg.T * 4.0 * G0 * G1 / (morph_ms * 1e-3) / 1e12
        peak = PEAK_F16_MFMA if scheme == "fp16" else PEAK_BF16_MFMA
        res["scheme"] = scheme
        ks, tb = (G0 + 15) // 16, (G1 + 31) // 32
        ceil = grid_ceiling("ws2d", -(-N // 32) * cfg.T,
                            {"unit": "wave-step (32 samples, one Euler step)",
                             "x_per_lane": 8 * ks, "y_per_lane": 16 * tb,
                             "mfma": 2 * nprod * ks * tb}) if scheme == "fp16" else None
        if ceil:
            ceil["frac"] = ceil["ceiling_ms"] / morph_ms
        # the unordered kernel on the same batch, for reference (same bits)
        P.morph_samples(occ, x0, cfg.T, cfg.eta, out=x1)
        e = Timer(torch)
        with e:
            P.morph_samples(occ, x0, cfg.T, cfg.eta, out=x1)
        res["unordered_kernel"] = {"kernel": "k_grid2d_mfma<2,4,kMorph>", "kernel_ms": e.ms(),
                                   "note": "the plain morph without the spatial order; the "
                                           "same bits per sample"}
        res["roofline"] = {"bound": "mfma", "achieved": fp32_tf, "peak": peak / 1e12,
                           "unit": "TFLOP/s", "frac": fp32_tf * 1e12 / peak,
                           "traffic": grid2d_traffic(),
                           "kernel": "k_grid2d_sorted<2,4> (after the 32x32-cell counting sort, "
                                     "timed with it)",
                           "kernel_ms": morph_ms, "kernel_ms_median": morph_median,
                           "skipping": "each wave skips the 16-hinge blocks and 8-row groups "
                                       "whose terms are exact zeros for all its samples; the "
                                       "work counted is the dense sum's",
                           "split_scheme": scheme,
                           "work": "4*G0*G1 FP32-accurate flops per sample-step (64x64 grid): "
                                   "the two G1 x G0 contractions, on "
                                   f"{scheme.upper()} MFMA as {nprod} split products each",
                           "mfma_issue": {"products_per_multiply_add": nprod,
                                          "achieved": nprod * fp32_tf,
                                          "frac": nprod * fp32_tf * 1e12 / peak},
                           "frac_ceiling_of_split_scheme": 1.0 / nprod,
                           "ceiling": ceil,
                           "instruction_counts": grid2d_counts(),
                           "traffic_note": "HBM bytes per call, the sort's kernels included "
                                           "(rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                           "copy-calibrated); algorithmic "
                                           f"{N * 2 * 4 * 2} bytes of state in and out, "
                                           f"{N * 2 * 4 * 4 + N * 4 * 2} with the sort's "
                                           "two reads of the batch, its permutation "
                                           "written and read"}
        # the pairwise kernel on the same batch, for reference
        dense = P.Occupancy(occ.hinges, occ.weights, occ.lengthscale)
        P.morph_samples(dense, x0, cfg.T, cfg.eta, out=x1)
        e = Timer(torch)
        with e:
            P.morph_samples(dense, x0, cfg.T, cfg.eta, out=x1)
        dms = e.ms()
        pairs = N * cfg.T * cfg.n_hinges
        ach = pairs * FLOPS_PER_PAIR[2] / (dms * 1e-3) / 1e12
        res["pairwise"] = {"kernel": "k_rbf<2,2,1,1024,kMorph>", "kernel_ms": dms,
                           "samples_per_s": N / (dms * 1e-3),
                           "roofline": {"bound": "alu", "achieved": ach,
                                        "peak": alu_peak_tflops(2), "unit": "TFLOP/s",
                                        "frac": ach / alu_peak_tflops(2)}}
        log(f"pairwise kernel on the same batch: {dms:.3f} ms")
    else:
        pairs = N * cfg.T * cfg.n_hinges
        achieved = pairs * FLOPS_PER_PAIR[2] / (morph_ms * 1e-3) / 1e12
        res["roofline"] = {"bound": "alu", "achieved": achieved, "peak": alu_peak_tflops(2),
                           "unit": "TFLOP/s", "frac": achieved / alu_peak_tflops(2),
                           "traffic": None, "kernel": "k_rbf<2,2,1,1024,kMorph>",
                           "kernel_ms": morph_ms,
                           "work": "12 FP32 flops + 1 exp per sample-hinge pair"}
    return res


def small_2d(P, I, K, torch, dev):
    cfg = K.C1
    sc = ws_scene(P, I, K, torch, cfg, dev)
    x0 = P.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, cfg.n_samples)
    x1 = torch.empty_like(x0)
    for _ in range(3):
        P.morph_samples(sc["occ"], x0, cfg.T, cfg.eta, out=x1)
    t = Timer(torch)
    reps = 20
    with t:
        for _ in range(reps):
            P.morph_samples(sc["occ"], x0, cfg.T, cfg.eta, out=x1)
    ms = t.ms() / reps
    _, h0 = P.label_points_discs(*sc["discs"], x0, count=True)
    _, h1 = P.label_points_discs(*sc["discs"], x1, count=True)
    return {"workload": "plain morph 2-D small: 4096 samples, 30x30 hinges, l=0.7, T=20, "
                        "eta=0.05, 20 discs",
            "morph_ms": ms, "samples_per_s": cfg.n_samples / (ms * 1e-3),
            "collision_free_before": 1 - h0.item() / cfg.n_samples,
            "collision_free_after": 1 - h1.item() / cfg.n_samples, "fit_ms": sc["fit_ms"]}


def arm_world(P, I, K, torch, dev):
    """7-DOF arm, box world, and the 3-D occupancy fitted on the GPU (config 4)."""
    c3, c4 = K.C3, K.C4
    a, d, al, th = I.dh_params(c3.cfg_id, c3.n_dof, c3.link_min, c3.link_max, c3.alpha)
    arm = P.Arm(a, d, al, th, c3.pts_per_link)
    bc, be = I.boxes(c3.cfg_id, c3.n_boxes, c3.box_lo, c3.box_hi, c3.half_min, c3.half_max)
    bc_d, be_d = torch.from_numpy(bc).to(dev), torch.from_numpy(be).to(dev)
    h = torch.from_numpy(I.hinge_grid(3, c3.grid, c3.box_lo, c3.box_hi)).to(dev)
    pts = torch.from_numpy(I.uniform_points(c4.cfg_id, K.STREAM_FIT, 3, c4.n_points, c3.box_lo,
                                            c3.box_hi)).to(dev)
    y = P.label_points_boxes(bc_d, be_d, pts)
    M = h.shape[1]
    w = torch.zeros(M + 1, dtype=torch.float32, device=dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    t = Timer(torch)
    with t:
        loss = P.fit_occupancy(h, c3.lengthscale, w, pts, y, c4.steps, c4.lr, c4.l2, "adam",
                               beta1=c4.beta1, beta2=c4.beta2, eps=c4.eps, adam_m=m, adam_v=v,
                               grid=(c3.grid,) * 3)
    fit_ms = t.ms()
    n = c4.n_points
    fit = {"workload": "occupancy fit 3-D: 2^20 labelled points, 16^3 hinges, l=0.15, BCE + "
                       "L2 1e-4, 500 full-batch Adam steps",
           "ms_total": fit_ms, "ms_per_step": fit_ms / c4.steps,
           "loss_first": float(loss[0]), "loss_last": float(loss[-1]),
           "pairs_per_s": 2.0 * n * M * c4.steps / (fit_ms * 1e-3)}
    occ = P.Occupancy(h, w, c3.lengthscale, grid=(c3.grid,) * 3)
    return dict(arm=arm, boxes=(bc_d, be_d), occ=occ, fit=fit)


def arm_morph(P, I, K, torch, world):
    c3 = K.C3
    arm, occ = world["arm"], world["occ"]
    q0 = P.uniform_samples(I.philox_seed(c3.cfg_id), 0, [c3.q_lo] * 7, [c3.q_hi] * 7, c3.n_samples)
    q1 = torch.empty_like(q0)
    P.morph_samples(occ, q0, c3.T, c3.eta, arm=arm, out=q1)
    t = Timer(torch)
    reps = 3
    with t:
        for _ in range(reps):
            P.morph_samples(occ, q0, c3.T, c3.eta, arm=arm, out=q1)
    ms = t.ms() / reps
    _, h0 = P.label_configs(arm, *world["boxes"], q0, count=True)
    _, h1 = P.label_configs(arm, *world["boxes"], q1, count=True)
    # algorithmic work of the factorised evaluation per body point and step: two
    # (16*16) x 16 matrix-vector products = 4 * 4096 FP32 flops, on the matrix cores at
    # FP32 accuracy as the split scheme's products (three FP16 or six BF16)
    scheme, nprod = P.split_scheme(occ)
    peak = PEAK_F16_MFMA if scheme == "fp16" else PEAK_BF16_MFMA
    fp32_tf = c3.n_samples * c3.T * c3.n_body * 4.0 * c3.n_hinges / (ms * 1e-3) / 1e12
    ceil = grid_ceiling("arm", (c3.n_samples // 4) * c3.T * c3.n_dof,
                        {"unit": "wave link-step (4 configurations x 8 body points, one "
                                 "link, one step)",
                         "x_per_lane": 8, "y_per_lane": 8, "z_per_lane": 16,
                         "contraction_fma_per_lane": 8 * 56,
                         "mfma": 2 * nprod * 8}) if scheme == "fp16" else None
    if ceil:
        ceil["frac"] = ceil["ceiling_ms"] / ms
    res = {"workload": "plain morph 7-DOF arm: 65,536 configurations, 56 body points, 16^3 "
                       "hinges, l=0.15, T=30, eta=0.01, 40 boxes",
           "morph_ms": ms, "samples_per_s": c3.n_samples / (ms * 1e-3),
           "collision_free_before": 1 - h0.item() / c3.n_samples,
           "collision_free_after": 1 - h1.item() / c3.n_samples,
           "roofline": {"bound": "mfma", "achieved": fp32_tf, "peak": peak / 1e12,
                        "unit": "TFLOP/s", "frac": fp32_tf * 1e12 / peak,
                        "kernel": "k_arm_grid3d<7,16,16,true>", "split_scheme": scheme,
                        "work": "4*M FP32-accurate flops per body point and step (the two "
                                f"contractions), on {scheme.upper()} MFMA as {nprod} split "
                                "products each",
                        "mfma_issue": {"products_per_multiply_add": nprod,
                                       "achieved": nprod * fp32_tf,
                                       "frac": nprod * fp32_tf * 1e12 / peak},
                        "frac_ceiling_of_split_scheme": 1.0 / nprod,
                        "ceiling": ceil}}
    dense = P.Occupancy(occ.hinges, occ.weights, occ.lengthscale)
    P.morph_samples(dense, q0, c3.T, c3.eta, arm=arm, out=q1)
    t = Timer(torch)
    with t:
        P.morph_samples(dense, q0, c3.T, c3.eta, arm=arm, out=q1)
    dms = t.ms()
    pairs = c3.n_samples * c3.T * c3.n_body * c3.n_hinges
    a2 = pairs * FLOPS_PER_PAIR[3] / (dms * 1e-3) / 1e12
    res["pairwise_kernel"] = {"kernel": "k_morph_arm<7,512>", "morph_ms": dms,
                              "samples_per_s": c3.n_samples / (dms * 1e-3),
                              "roofline": {"bound": "alu", "achieved": a2,
                                           "peak": alu_peak_tflops(3), "unit": "TFLOP/s",
                                           "frac": a2 / alu_peak_tflops(3)}}
    return res


def tanh_morph(P, I, K, torch, dev):
    """The morph of the large 2-D workload with the paper's own occupancy, the tanh
    network of Sec. 3.1, fitted on the GPU first (full-batch Adam on the BCE)."""
    cfg, tc = K.C2, K.TANH
    H, L = tc.hidden, tc.layers
    dc, dr = I.discs(cfg.cfg_id, cfg.n_discs, cfg.lo, cfg.hi, cfg.r_min, cfg.r_max)
    dc_d, dr_d = torch.from_numpy(dc).to(dev), torch.from_numpy(dr).to(dev)
    pts = torch.from_numpy(I.uniform_points(cfg.cfg_id, K.STREAM_FIT, 2, cfg.fit_points, cfg.lo,
                                            cfg.hi)).to(dev)
    y = P.label_points_discs(dc_d, dr_d, pts)
    init = torch.from_numpy(I.tanh_init(cfg.cfg_id, 2, H, L, cfg.hi)).to(dev)
    net = P.TanhNet(2, H, L, init)
    t = Timer(torch)
    with t:
        loss = P.tanh_fit(net, pts, y, tc.steps[1], tc.lr, tc.l2[1], tc.beta1, tc.beta2, tc.eps)
    fit_ms = t.ms()
    log(f"tanh-network fit: {fit_ms:.0f} ms, loss {float(loss[0]):.4f} -> {float(loss[-1]):.4f}")
    N = cfg.n_samples
    x0 = P.uniform_samples(I.philox_seed(cfg.cfg_id), 0, [cfg.lo] * 2, [cfg.hi] * 2, N)
    x1 = torch.empty_like(x0)
    P.tanh_morph_samples(net, x0, cfg.T, cfg.eta, out=x1)
    reps = 3
    t = Timer(torch)
    with t:
        for _ in range(reps):
            P.tanh_morph_samples(net, x0, cfg.T, cfg.eta, out=x1)
    ms = t.ms() / reps
    _, h0 = P.label_points_discs(dc_d, dr_d, x0, count=True)
    _, h1 = P.label_points_discs(dc_d, dr_d, x1, count=True)
    # hidden-to-hidden products forward (W a) and backward (W^T e) on MFMA:
    # 4 (L-1) H^2 flops per sample and step; the forward half takes the scheme the
    # library reports (FP16 parts: 3 products, BF16: 6), the backward half 6 products
    scheme, fwd_products = P.tanh_split_scheme(net)
    products = (fwd_products + 6) / 2.0
    flops = N * cfg.T * 4.0 * (L - 1) * H * H
    ach = flops / (ms * 1e-3) / 1e12
    return {"workload": f"plain morph 2-D large with the paper's tanh occupancy (2-{H}x{L}-1, "
                        f"sigmoid): 1,048,576 samples, T={cfg.T}, eta={cfg.eta}, 100 discs",
            "fit": {"steps": tc.steps[1], "points": cfg.fit_points, "ms_total": fit_ms,
                    "loss_first": float(loss[0]), "loss_last": float(loss[-1])},
            "morph_ms": ms, "samples_per_s": N / (ms * 1e-3),
            "collision_free_before": 1 - h0.item() / N,
            "collision_free_after": 1 - h1.item() / N,
            "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16_MFMA / 1e12,
                         "unit": "TFLOP/s", "frac": ach * 1e12 / PEAK_BF16_MFMA,
                         "kernel": f"k_tanh_net<2,4,{L},kMorph>",
                         "work": "4*(L-1)*H^2 FP32-accurate flops per sample-step (the forward "
                                 "and backward hidden products): the forward on the reported "
                                 "scheme's parts, the backward on six BF16 products of three-way "
                                 "splits",
                         "forward_scheme": scheme,
                         "mfma_issue": {"products_per_multiply_add": products,
                                        "achieved": products * ach,
                                        "frac": products * ach * 1e12 / PEAK_BF16_MFMA},
                         "frac_ceiling_of_split_scheme": 1.0 / products}}


def density_workload(P, I, K, torch, hl):
    """Log-determinant of the morph, its inverse by fixed point and the epsilon
    mixture on the large 2-D workload (same occupancy and prior batch as the headline)."""
    cfg = K.C2
    occ, x0, N = hl["sc"]["occ"], hl["x0"], hl["N"]
    G0 = G1 = cfg.grid
    out = torch.empty_like(x0)
    iters = 10
    # the unordered kernels, then the ordered calls (counting sort + exact-zero
    # skipping, the sort timed with them) that must give the same bits
    P.morph_logdet(occ, x0, cfg.T, cfg.eta, out=out)
    t = Timer(torch)
    with t:
        _, ld_u = P.morph_logdet(occ, x0, cfg.T, cfg.eta, out=out)
    ld_u_ms = t.ms()
    t = Timer(torch)
    with t:
        y_u, ld_inv_u, resid_u = P.morph_inverse(occ, out, cfg.T, cfg.eta, iters)
    inv_u_ms = t.ms()
    ws = P.morph_workspace(occ, N, cfg.T)
    out_o = torch.empty_like(x0)
    P.morph_logdet(occ, x0, cfg.T, cfg.eta, out=out_o, ordered=True, ws=ws)
    t = Timer(torch)
    with t:
        _, ld = P.morph_logdet(occ, x0, cfg.T, cfg.eta, out=out_o, ordered=True, ws=ws)
    ld_ms = t.ms()
    t = Timer(torch)
    with t:
        y, ld_inv, resid = P.morph_inverse(occ, out, cfg.T, cfg.eta, iters, ordered=True, ws=ws)
    inv_ms = t.ms()
    same_bits = bool(torch.equal(out_o, out) and torch.equal(ld, ld_u) and torch.equal(y, y_u)
                     and torch.equal(ld_inv, ld_inv_u) and torch.equal(resid, resid_u))
    rt = (y - x0).abs().amax(dim=0)
    ldd = (ld_inv - ld).abs().max().item()
    seed = I.philox_seed(cfg.cfg_id)
    eps = 0.1
    P.mixture_samples(occ, seed, 7, [cfg.lo] * 2, [cfg.hi] * 2, N, eps, cfg.T, cfg.eta)
    t = Timer(torch)
    with t:
        _, mixed, keep = P.mixture_samples(occ, seed, 7, [cfg.lo] * 2, [cfg.hi] * 2, N, eps,
                                           cfg.T, cfg.eta)
    mix_ms = t.ms()
    dc_d, dr_d = hl["sc"]["discs"]
    _, hm = P.label_points_discs(dc_d, dr_d, mixed, count=True)
    # U, V, Q products (6 G0 G1 FP32-equivalent flops) per sample-step on the logdet
    # path, each multiply-add as the split scheme's products (three FP16 or six BF16)
    scheme, nprod = P.split_scheme(occ)
    peak = PEAK_F16_MFMA if scheme == "fp16" else PEAK_BF16_MFMA
    sname = scheme.upper()
    ach = N * cfg.T * 6.0 * G0 * G1 / (ld_ms * 1e-3) / 1e12
    inv_flops = N * cfg.T * (iters * 4.0 + 6.0) * G0 * G1
    return {"workload": "log-det, inverse (fixed point, 10 iterations per step) and epsilon "
                        "mixture (eps=0.1) of the 2-D large morph: 1,048,576 samples, 64x64 "
                        "hinges, T=50, eta=0.02",
            "path": "ordered (pdmp_morph_logdet_ws, pdmp_morph_inverse_ws: counting sort, "
                    "then exact-zero skipping; the sort included in the times)",
            "logdet_ms": ld_ms, "logdet_samples_per_s": N / (ld_ms * 1e-3),
            "inverse_ms": inv_ms, "inverse_samples_per_s": N / (inv_ms * 1e-3),
            "unordered": {"logdet_ms": ld_u_ms, "inverse_ms": inv_u_ms,
                          "same_bits_as_ordered": same_bits},
            "inverse_residual_max": resid.max().item(),
            "round_trip_err_max": rt.max().item(), "round_trip_err_median": rt.median().item(),
            "logdet_roundtrip_diff_max": ldd,
            "logdet_mean": ld.mean().item(),
            "mixture_ms": mix_ms, "mixture_kept_fraction": keep.float().mean().item(),
            "mixture_collision_free": 1 - hm.item() / N,
            "roofline_logdet": {"bound": "mfma", "achieved": ach,
                                "peak": peak / 1e12, "unit": "TFLOP/s",
                                "frac": ach * 1e12 / peak,
                                "kernel": "k_grid2d_inv_sorted<2,4,kLogdet> (sort included)",
                                "split_scheme": scheme,
                                "work": "6*G0*G1 FP32-accurate flops per sample-step (the three "
                                        f"contractions), on {sname} MFMA as {nprod} split "
                                        "products each",
                                "mfma_issue_frac": nprod * ach * 1e12 / peak},
            "roofline_inverse": {"bound": "mfma",
                                 "achieved": inv_flops / (inv_ms * 1e-3) / 1e12,
                                 "peak": peak / 1e12, "unit": "TFLOP/s",
                                 "frac": inv_flops / (inv_ms * 1e-3) / peak,
                                 "kernel": "k_grid2d_inv_sorted<2,4,kInverse> (sort included)",
                                 "split_scheme": scheme,
                                 "work": "(4*iters + 6)*G0*G1 FP32-accurate flops per "
                                         f"sample-step, on {sname} MFMA as {nprod} split "
                                         "products each",
                                 "mfma_issue_frac": nprod * inv_flops / (inv_ms * 1e-3) / peak}}


def pipeline_workload(args, P, I, K, torch, dev, hl):
    """The producer/consumer of Sec. 3.3: a background GPU sampler filling the bucket,
    a plane RRT drawing from it (prior when empty).  (a) the morphed share of the
    consumed samples over time and the producer's delivered rate in config 2's world;
    (b) with --rrt-runs R, the plane RRT's time to solution in config 1's world with the
    morph sampler against the prior, R runs each (a planner comparison, off by
    default)."""
    import numpy as np
    out = {}
    c1 = K.C1
    dc1, dr1 = I.discs(c1.cfg_id, c1.n_discs, c1.lo, c1.hi, c1.r_min, c1.r_max)
    start, goal = K.RRT_START_GOAL[1]
    runs = {"prior": [], "morph": []}
    sc1 = ws_scene(P, I, K, torch, c1, dev) if args.rrt_runs > 0 else None
    for r in range(args.rrt_runs):
        for kind in ("prior", "morph"):
            s = P.Sampler(sc1["occ"] if kind == "morph" else None, 2, [c1.lo] * 2, [c1.hi] * 2,
                          c1.T, c1.eta, c1.n_samples, 1 << 16, seed=I.philox_seed(c1.cfg_id),
                          stream_id=1000 * r, prior_stream_id=50 + r)
            if kind == "morph":
                s.start()
            res = P.rrt_run(s, start, goal, 0.5, 0.5, (dc1, dr1), 200000, 5.0)
            runs[kind].append({"solved": res["solved"], "iters": res["iters"],
                               "nodes": res["n_nodes"], "s": res["elapsed_s"],
                               "from_bucket": res["from_bucket"], "path_len": res["path_len"]})
            s.close()
    for kind, rs in runs.items():
        if not rs:
            continue
        ok = [x for x in rs if x["solved"]]
        out[f"config1_{kind}"] = {
            "solved": len(ok), "runs": len(rs),
            "iters_mean": float(np.mean([x["iters"] for x in ok])) if ok else None,
            "seconds_mean": float(np.mean([x["s"] for x in ok])) if ok else None,
            "path_len_mean": float(np.mean([x["path_len"] for x in ok])) if ok else None,
            "morphed_share": float(np.sum([x["from_bucket"] for x in rs]) /
                                   max(1, np.sum([x["iters"] for x in rs])))}
    c2 = K.C2
    dc2, dr2 = hl["sc"]["discs"]
    s = P.Sampler(hl["sc"]["occ"], 2, [c2.lo] * 2, [c2.hi] * 2, c2.T, c2.eta, 65536, 1 << 20,
                  seed=I.philox_seed(c2.cfg_id), stream_id=5000, prior_stream_id=77)
    s.start()
    start2, goal2 = K.RRT_START_GOAL[2]
    res = P.rrt_run(s, start2, goal2, 0.5, -1.0, (dc2.cpu().numpy(), dr2.cpu().numpy()),
                    3_000_000, 1.0)
    st = s.stats()
    s.close()
    t, fb = res["t_sample"], res["sample_from_bucket"].astype(np.int64)
    share = []
    for cp in (0.001, 0.002, 0.005, 0.01, 0.02, 0.05, 0.1, 0.2, 0.5, 1.0):
        k = int(np.searchsorted(t, cp, side="right"))
        nb = int(fb[:k].sum())
        share.append({"t_s": cp, "from_bucket": nb, "from_prior": k - nb})
    out["config2_share_over_time"] = share
    out["config2_consumer"] = {"iters": res["iters"], "nodes": res["n_nodes"],
                               "from_bucket": res["from_bucket"], "from_prior": res["from_prior"],
                               "seconds": res["elapsed_s"]}
    out["config2_producer_during_run"] = {"batches": st["batches"], "produced": st["produced"],
                                          "status": st["status"]}
    # the producer alone: time to fill an empty bucket of 2^23 samples
    cap = 1 << 23
    s = P.Sampler(hl["sc"]["occ"], 2, [c2.lo] * 2, [c2.hi] * 2, c2.T, c2.eta, 65536, cap,
                  seed=I.philox_seed(c2.cfg_id), stream_id=9000, prior_stream_id=78)
    t0 = time.perf_counter()
    s.start()
    while s.stats()["produced"] < cap and time.perf_counter() - t0 < 10.0:
        time.sleep(0.0005)
    dt = time.perf_counter() - t0
    st = s.stats()
    s.close()
    out["producer"] = {"produced": st["produced"], "seconds": dt,
                       "samples_per_s": st["produced"] / dt, "status": st["status"],
                       "note": "morph (T=50, 65,536-sample batches) + PCIe copy to pinned host "
                               "memory + push into the bucket, from thread start to a full "
                               "2^23-sample bucket"}
    return out


def culled_workload(P, I, K, torch, hl):
    """Compact-support hinge culling (a variant beyond the paper) on the large 2-D
    workload: each point takes the hinges of the 3x3 cells (side >= 5.5 l) around it."""
    import numpy as np
    cfg = K.C2
    occ, x0, N = hl["sc"]["occ"], hl["x0"], hl["N"]
    dense = P.Occupancy(occ.hinges, occ.weights, occ.lengthscale)
    rc = 5.5 * cfg.lengthscale
    g = P.cull_grid(2, [cfg.lo] * 2, [cfg.hi] * 2, rc)
    out = torch.empty_like(x0)
    P.morph_culled(dense, g, x0, cfg.T, cfg.eta, out=out)
    t = Timer(torch)
    reps = 3
    with t:
        for _ in range(reps):
            P.morph_culled(dense, g, x0, cfg.T, cfg.eta, out=out)
    ms = t.ms() / reps
    # own work: the pairs of each point with the hinges of its 3x3 cells, counted at the
    # start and at the end of the path (the mean of the two stands for every step)
    h = occ.hinges.cpu().numpy().astype(np.float64)
    nc = [g.nc[0], g.nc[1]]
    inv = float(g.inv_cell)

    def cells(v, k):
        c = np.floor((v.astype(np.float64) - float(g.lo[k])) * inv)
        return np.clip(c, 0, nc[k] - 1).astype(np.int64)

    hc = np.zeros((nc[1] + 2, nc[0] + 2), np.int64)
    np.add.at(hc, (cells(h[1], 1) + 1, cells(h[0], 0) + 1), 1)
    box = sum(np.roll(np.roll(hc, dy, 0), dx, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))

    def pairs(x):
        xn = x.cpu().numpy()
        return float(box[cells(xn[1], 1) + 1, cells(xn[0], 0) + 1].mean())

    per_point = 0.5 * (pairs(x0) + pairs(out))
    flops = N * cfg.T * per_point * FLOPS_PER_PAIR[2]
    ach = flops / (ms * 1e-3) / 1e12
    dc_d, dr_d = hl["sc"]["discs"]
    _, h1 = P.label_points_discs(dc_d, dr_d, out, count=True)
    ref = P.morph_samples(dense, x0, cfg.T, cfg.eta)
    dev_max = (ref - out).abs().amax(dim=0)
    W = float(occ.weights[:-1].abs().sum())
    return {"workload": "culled pairwise morph 2-D large: 1,048,576 samples, 64x64 hinges, "
                        "l=0.4, cutoff 5.5 l (3x3 cells of side 2.2), T=50, eta=0.02",
            "morph_ms": ms, "samples_per_s": N / (ms * 1e-3),
            "pairs_per_point_step": per_point, "dense_pairs_per_point_step": cfg.n_hinges,
            "logit_tail_bound": W * float(np.exp(-rc * rc / (2 * cfg.lengthscale ** 2))),
            "max_dev_from_dense_morph": dev_max.max().item(),
            "median_dev_from_dense_morph": dev_max.median().item(),
            "collision_free_after": 1 - h1.item() / N,
            "roofline": {"bound": "alu", "achieved": ach, "peak": alu_peak_tflops(2),
                         "unit": "TFLOP/s", "frac": ach / alu_peak_tflops(2),
                         "kernel": "k_cull_morph<2>",
                         "work": "12 FP32 flops + 1 exp per kept (point, hinge) pair, own "
                                 "culled pairs only"}}


AMORTISED_VARIANTS = (
    # name, epochs factor, schedule, hard weight, threshold that marks a sample hard
    ("hard x4 at 0.1", 1, None, 4.0, 0.1),
    ("hard x16 at 0.1", 1, None, 16.0, 0.1),
    ("3x epochs, cosine with 4 restarts", 3, "cosine_restarts", None, None),
)
AMORTISED_THRESHOLDS = (0.5, 0.3, 0.2, 0.1, 0.05, 0.02)
# the refining variant: trigger thresholds x plain steps from q_hat
REFINE_POINTS = tuple((th, tr) for th in (0.1, 0.07, 0.05, 0.03) for tr in (6, 7, 8, 9, 10, 12))


def amortised_frontier(P, K, torch, world, mlp, q, pl_ms, cf_plain, refine=False):
    """Fallback fraction, collision-free fraction and speedup over the plain morph at each
    trigger threshold (with refine: at each threshold and refining step count), and the
    fastest point within one point of the plain morph's collision-free fraction."""
    c3 = K.C3
    arm, occ = world["arm"], world["occ"]
    n = int(q.shape[1])
    points = REFINE_POINTS if refine else tuple((th, c3.T) for th in AMORTISED_THRESHOLDS)
    sweep = []
    for th, steps in points:
        o2, f2, n2 = P.amortised_morph(mlp, occ, arm, q, steps, c3.eta, th, refine=refine)
        ms2 = median_ms(torch, lambda: P.amortised_morph(mlp, occ, arm, q, steps, c3.eta, th,
                                                         out=o2, flag=f2, n_fallback=n2,
                                                         refine=refine))
        _, h2 = P.label_configs(arm, *world["boxes"], o2, count=True)
        r = {"threshold": th, "ms": ms2, "speedup": pl_ms / ms2,
             "fallback_fraction": int(n2.item()) / n, "collision_free": 1 - h2.item() / n}
        if refine:
            r["refine_steps"] = steps
        sweep.append(r)
    eq = [r for r in sweep if r["collision_free"] >= cf_plain - 0.01]
    return sweep, (max(eq, key=lambda r: r["speedup"]) if eq else None)


def amortised(args, P, I, K, torch, world):
    from paper_2108_11775_amd import amortise
    c3, c5 = K.C3, K.C5
    arm, occ = world["arm"], world["occ"]
    n_batches = args.train_batches or c5.train_pairs // c5.batch
    epochs = args.train_epochs or c5.epochs
    t = Timer(torch)
    with t:
        pairs = amortise.make_pairs(occ, arm, n_batches, c5.batch, c3.T, c3.eta,
                                    I.philox_seed(c5.cfg_id), c3.q_lo, c3.q_hi)
    gen_ms = t.ms()
    log(f"training pairs: {n_batches} x {c5.batch} in {gen_ms / 1e3:.1f} s")

    def trained(ep, schedule, hard_weight, hard_thresh):
        mlp = P.Mlp.from_layers(I.mlp_init(c5.cfg_id, c5.widths))
        t = Timer(torch)
        with t:
            losses = amortise.train(mlp, pairs, ep, c5.lr, c5.beta1, c5.beta2, c5.eps, log=log,
                                    schedule=schedule, hard_weight=hard_weight, occ=occ,
                                    arm=arm, hard_thresh=hard_thresh or 0.5)
        return mlp, losses, t.ms()

    mlp, losses, train_ms = trained(epochs, c5.schedule, None, None)
    variant_nets = []
    if args.amortised_variants:
        for name, fac, sched, hw, hth in AMORTISED_VARIANTS:
            log(f"amortised variant: {name}")
            vm, vl, vms = trained(epochs * fac, sched or c5.schedule, hw, hth)
            variant_nets.append((name, fac, sched or c5.schedule, hw, hth, vm, vl, vms))
    del pairs
    q = P.uniform_samples(I.philox_seed(c5.cfg_id, K.STREAM_EVAL), 0, [c3.q_lo] * 7,
                          [c3.q_hi] * 7, c5.eval_samples)
    out, flag, nf = P.amortised_morph(mlp, occ, arm, q, c3.T, c3.eta, c5.threshold)
    reps = 5
    t = Timer(torch)
    with t:
        for _ in range(reps):
            P.amortised_morph(mlp, occ, arm, q, c3.T, c3.eta, c5.threshold, out=out, flag=flag,
                              n_fallback=nf)
    am_ms = t.ms() / reps
    plain_out = P.morph_samples(occ, q, c3.T, c3.eta, arm=arm)
    pl_ms = median_ms(torch, lambda: P.morph_samples(occ, q, c3.T, c3.eta, arm=arm,
                                                     out=plain_out))
    _, ha = P.label_configs(arm, *world["boxes"], out, count=True)
    _, hp = P.label_configs(arm, *world["boxes"], plain_out, count=True)
    _, h0 = P.label_configs(arm, *world["boxes"], q, count=True)
    zero = P.Mlp.from_layers(I.mlp_init(c5.cfg_id, c5.widths))
    _, fz, nz = P.amortised_morph(zero, occ, arm, q, c3.T, c3.eta, c5.threshold)
    n = c5.eval_samples
    nf_v = int(nf.item())
    # operating point at an equal collision-free fraction (within 1 point of the plain
    # morph's): the fastest threshold of the sweep that reaches it
    cf_plain = 1 - hp.item() / n
    sweep, equal_cf = amortised_frontier(P, K, torch, world, mlp, q, pl_ms, cf_plain)
    res = {"workload": "amortised morph: residual MLP 7-256-256-256-7 SiLU (BF16 MFMA, FP32 "
                       "accumulate) trained on plain-morph pairs, plain T=30 fallback where "
                       "max body-point occupancy > 0.5; 65,536 held-out configurations",
           "train_pairs": n_batches * c5.batch, "epochs": epochs,
           "pair_generation_s": gen_ms / 1e3, "train_s": train_ms / 1e3,
           "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
           "amortised_ms": am_ms, "amortised_samples_per_s": n / (am_ms * 1e-3),
           "plain_ms": pl_ms, "plain_samples_per_s": n / (pl_ms * 1e-3),
           "speedup": pl_ms / am_ms, "fallback_fraction": nf_v / n,
           "fallback_fraction_without_network": int(nz.item()) / n,
           "collision_free_prior": 1 - h0.item() / n,
           "collision_free_amortised": 1 - ha.item() / n,
           "collision_free_plain": cf_plain,
           "at_equal_collision_free": equal_cf,
           "threshold_sweep": sweep}
    # the refining variant: flagged configurations take a few plain steps from q_hat
    rs, re_ = amortised_frontier(P, K, torch, world, mlp, q, pl_ms, cf_plain, refine=True)
    res["refine_variant"] = {"fallback": "flagged configurations take refine_steps plain steps "
                                         "from q + f(q) instead of T from q",
                             "at_equal_collision_free": re_, "sweep": rs}
    if variant_nets:
        res["variants"] = []
        for name, fac, sched, hw, hth, vm, vl, vms in variant_nets:
            vs, ve = amortised_frontier(P, K, torch, world, vm, q, pl_ms, cf_plain)
            rvs, rve = amortised_frontier(P, K, torch, world, vm, q, pl_ms, cf_plain, refine=True)
            res["variants"].append({"variant": name, "epochs": epochs * fac, "schedule": sched,
                                    "hard_weight": hw, "hard_threshold": hth,
                                    "train_s": vms / 1e3, "loss_last": float(vl[-1]),
                                    "at_equal_collision_free": ve, "threshold_sweep": vs,
                                    "refine_at_equal_collision_free": rve, "refine_sweep": rvs})
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is designed, not built)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    names = ("small", "density", "culled", "pipeline", "tanh", "arm", "amortised")
    sel = set(names) if args.workloads == "all" else set(args.workloads.split(","))
    if sel - set(names):
        sys.exit(f"unknown workloads {sorted(sel - set(names))}; choose from {names}")
    import torch
    import paper_2108_11775_amd as P
    from paper_2108_11775_amd import configs as K, inputs as I

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 2 x 256 MiB device copies")
        del src, dst
    RATES.update(P.issue_rates())
    log("issue costs (cycles per wave64 instruction per SIMD): " +
        ", ".join(f"{k} {v:.2f}" for k, v in RATES.items()))
    hl = headline(args, P, I, K, torch, dev)
    cfg = hl["cfg"]
    out = {
        "metric": "morphed samples/s (T steps) + collision-free fraction; amortised vs plain morph",
        "value": hl["N"] / (hl["ms_step"] * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "clock_settle_s": args.settle_s,
        "ms_per_step": hl["ms_step"],
        "ms_per_step_median": hl["step_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+" + {"fp16": "f16x3", "bf16": "bf16x6"}.get(hl.get("scheme"), "f32"),
        "data": "synthetic (seeded disc world, Philox prior samples, occupancy fitted on the GPU)",
        "config": {"workload": "plain morph 2-D large: 1,048,576 samples, 64x64 hinges, "
                               "l=0.4, T=50, eta=0.02, 100 discs",
                   "N": hl["N"], "T": cfg.T, "M": cfg.n_hinges, "eta": cfg.eta,
                   "path": "grid factorisation (FP32-accurate split MFMA)" if hl["sc"]["occ"].grid else
                           "pairwise RBF sum"},
        "collision_free_before": hl["free_before"],
        "collision_free_after": hl["free_after"],
        "roofline": hl["roofline"],
        "issue_rates": {"cycles_per_wave64_instruction": {k: v for k, v in RATES.items()
                                                          if k != "clock_ghz"},
                        "probe_clock_ghz": RATES["clock_ghz"],
                        "source": "pdmp_issue_rates on this device, this run"},
    }
    if "pairwise" in hl:
        out["pairwise_kernel"] = hl["pairwise"]
    if "unordered_kernel" in hl:
        out["unordered_kernel"] = hl["unordered_kernel"]
    out["fit_ms"] = hl["sc"]["fit_ms"]
    world = None
    if not args.headline_only:
        wl = {}
        try:
            if "small" in sel:
                wl["ws2d_small"] = small_2d(P, I, K, torch, dev)
                log("small 2-D done")
            if "density" in sel and hl["sc"]["occ"].grid:
                wl["density_ws2d"] = density_workload(P, I, K, torch, hl)
                dw = wl["density_ws2d"]
                log(f"log-det / inverse, ordered: {dw['logdet_ms']:.2f} / {dw['inverse_ms']:.2f} "
                    f"ms (unordered {dw['unordered']['logdet_ms']:.2f} / "
                    f"{dw['unordered']['inverse_ms']:.2f} ms, same bits: "
                    f"{dw['unordered']['same_bits_as_ordered']})")
            if "culled" in sel:
                wl["culled_ws2d"] = culled_workload(P, I, K, torch, hl)
                log(f"culled morph: {wl['culled_ws2d']['morph_ms']:.2f} ms")
            if "pipeline" in sel:
                wl["pipeline"] = pipeline_workload(args, P, I, K, torch, dev, hl)
                log("producer/consumer done")
            if "tanh" in sel:
                wl["tanh_ws2d"] = tanh_morph(P, I, K, torch, dev)
                log(f"tanh-network morph: {wl['tanh_ws2d']['morph_ms']:.2f} ms")
            if "arm" in sel or "amortised" in sel:
                world = arm_world(P, I, K, torch, dev)
                wl["fit3d"] = world["fit"]
                log(f"3-D fit: {world['fit']['ms_total']:.0f} ms")
            if "arm" in sel:
                wl["arm7"] = arm_morph(P, I, K, torch, world)
                log(f"arm morph: {wl['arm7']['morph_ms']:.1f} ms")
            if "amortised" in sel:
                wl["amortised"] = amortised(args, P, I, K, torch, world)
                am = wl["amortised"]
                eq = am["at_equal_collision_free"]
                log(f"amortised: speedup {am['speedup']:.2f}x at threshold {K.C5.threshold}; "
                    "at equal collision-free fraction "
                    + (f"{eq['speedup']:.2f}x (threshold {eq['threshold']})" if eq
                       else "not reached"))
                rq = am["refine_variant"]["at_equal_collision_free"]
                log("refining variant at equal collision-free fraction: "
                    + (f"{rq['speedup']:.2f}x (threshold {rq['threshold']}, "
                       f"{rq['refine_steps']} steps)" if rq else "not reached"))
        except Exception as e:  # report what ran; the headline stands on its own
            wl["error"] = f"{type(e).__name__}: {e}"
        out["workloads"] = wl
    if not args.no_cpu_baseline:
        # the FP64 oracle on the host: the CPU baseline, and its one-step check along the
        # GPU paths of this run
        import oracle as O
        log("cpu baseline ...")
        P.uniform_samples(hl["seed"], 0, [cfg.lo] * 2, [cfg.hi] * 2, hl["N"], out=hl["x0"])
        x0_np = hl["x0"].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(O, hl["sc"]["h"], hl["sc"]["w"], cfg.lengthscale,
                                           x0_np, cfg, args.cpu_sample)
        if not args.no_trajectory_check:
            log("one-step check along the GPU paths ...")
            try:
                out["trajectory_check"] = trajectory_check(O, P, I, K, torch, hl, world)
            except Exception as e:  # reported, the headline stands on its own
                out["trajectory_check"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
