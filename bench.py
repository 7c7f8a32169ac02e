"""Benchmark: point*pixel/s of the hologram hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: a 1920 x 1080 hologram of 10,000 points (8 um pitch, 532 nm,
x, y ~ U(+-3 mm), z ~ U[0.5, 0.6] m, A ~ U[0, 1]; seeded synthetic cloud,
cghgen config 2), points resident in HBM before timing.  One step = one
cgh_compute of the whole cloud in the headline mode (BF16 hi/lo split on the
matrix cores: per-point constants, factor build, split GEMM, split-K reduce).
The direct FP32 kernel and the other modes are timed the same way and
reported under "modes" (spherical_fp32 evaluates the exact spherical wave of
Eq. (1) instead of the Fresnel sum).

Side measurements, each on its own workload: the 64-frame batch ("batch",
tuned, replayed as a graph), the phase-only hologram of Eq. (3) ("kinoform"),
the 2048 x 2048 and 4096 x 4096 clouds ("large"), the wavefront-recording
method at 1920 x 1080 with 10^3 .. 10^5 points ("wrm") and the Fresnel
diffraction of Eq. (10) at the paper's plane sizes ("fresnel_diffraction").

Every GPU measurement runs first, keeping host copies of its outputs on the
evaluation sets; the FP64 oracle then runs on the host alone: first the CPU
baseline (the oracle on every 3rd row of the headline workload, all host
cores, timed), which is also the reference of every mode's NRMS, then the
other legs' references -- every 8th row and column of the 2048^2 cloud and
of all 64 batch frames, the centred 256 x 256 crop of the 4096^2 cloud,
sampled rows of the recorded planes.

Prints one JSON line (rank 0).  --gpus N > 1 is refused: the benchmark
measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks (dense MFMA; HBM).
PEAK_MFMA_BF16_TFLOPS = 2500.0
PEAK_MFMA_FP16_TFLOPS = 2500.0
PEAK_MFMA_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
CUS, CLOCK_HZ = 256, 2.4e9
# ALU-bound kernels: an upper bound from two per-CU limits at the peak clock --
# VALU issue of 64 lane-instructions per clock (4 SIMD16 units, one wave64
# instruction per 4 clocks each; every instruction, transcendental or not,
# takes one such slot) and transcendental results (v_cos/v_sin/v_sqrt/v_rcp)
# at half that rate, 32 per clock.
VALU_PER_CLK, TRANS_PER_CLK = 64, 32


def alu_peak_pps(instr_per_pp: int, trans_per_pp: int) -> float:
    return CUS * CLOCK_HZ * min(VALU_PER_CLK / instr_per_pp, TRANS_PER_CLK / trans_per_pp)


# direct kernel: v_add_f32_dpp, v_cos_f32, v_fmac_f32 per point*pixel
PEAK_DIRECT_PPS = alu_peak_pps(3, 1)          # 1.311e13 point*pixel/s
# The same three instructions with the cosine holding its SIMD for two issue
# slots (it does not overlap its neighbours in this loop; the kernel's VALU
# counters then read 95 % busy): 4 slots per point*pixel.
PEAK_DIRECT_ISSUE_PPS = CUS * CLOCK_HZ * VALU_PER_CLK / 4      # 9.830e12 point*pixel/s
# exact spherical wave: 2 v_add_f32_dpp, 2 v_add_f32, 2 v_mul_f32, v_fma_f32,
# v_fmac_f32 and v_sqrt_f32, v_rcp_f32, v_cos_f32 per point*pixel
PEAK_SPHERE_PPS = alu_peak_pps(11, 3)         # 3.575e12 point*pixel/s
# wavefront recording, per point*sample pair inside a disc: the FP64 disc test
# (v_add_f64 and v_cmp_le_f64; FP64 arithmetic issues at the FP32 rate here,
# v_fma_f64 57 lane-operations per clock per CU in the microbenchmark), two
# v_cndmask_b32 and four v_fma_f32 -- 8 slots; the line terms' cosines are per
# point and line, not per pair
PEAK_WRM_PAIRS = CUS * CLOCK_HZ * VALU_PER_CLK / 8              # 4.915e12 pairs/s
# FP32 vector arithmetic without packed operations: one multiply-add (2 flop)
# per lane and issue slot
PEAK_FP32_VALU_TFLOPS = CUS * CLOCK_HZ * VALU_PER_CLK * 2 / 1e12   # 78.6 TFLOP/s
ALU_MODES = {"direct_fp32": ("direct_fp32", PEAK_DIRECT_PPS),
             "spherical_fp32": ("direct_sphere", PEAK_SPHERE_PPS)}

# executed matrix flops per point*pixel: K = 2N columns, 2 flop per MAC, x products
FLOP_PER_PP = {"split_bf16": 12, "split_fp16": 12, "fp16": 4, "separable_fp32": 4}
GEMM_KERNEL = {"split_bf16": "gemm_split_mfma", "split_fp16": "gemm_split_mfma",
               "fp16": "gemm_mfma", "separable_fp32": "gemm_fp32_mfma"}
GEMM_PEAK = {"split_bf16": PEAK_MFMA_BF16_TFLOPS, "split_fp16": PEAK_MFMA_FP16_TFLOPS,
             "fp16": PEAK_MFMA_FP16_TFLOPS, "separable_fp32": PEAK_MFMA_FP32_TFLOPS}
MODE_DTYPE = {"split_bf16": "bf16", "split_fp16": "f16", "fp16": "f16", "direct_fp32": "f32",
              "separable_fp32": "f32", "spherical_fp32": "f32"}

# HBM bytes per launch from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch) over `python bench.py --traffic-driver`, each
# scaled by what the counter reads for a plain 256 MiB device copy (FETCH_SIZE
# reads half the true bytes: x2.0; WRITE_SIZE the true bytes: x1.0); see
# profiles/.  An entry holds for the kernel source it was taken on (sha256
# prefix) and its launch shape; otherwise the bench reports traffic null.
TRAFFIC_SCALE = {"fetch": 2.0, "write": 1.0}
TRAFFIC = [
    {"kernel": "gemm_split_mfma", "plan": "384,192,4,2,2,8", "src": "paper_1309_2734_amd/csrc/gemm.hip",
     "sha": "84eae018c8c7908b", "fetch_kib": 120352.9, "write_kib": 64800.3},
    {"kernel": "gemm_split_mfma", "plan": "192,384,2,4,2,8", "src": "paper_1309_2734_amd/csrc/gemm.hip",
     "sha": "84eae018c8c7908b", "fetch_kib": 120349.0, "write_kib": 64801.1},
    # 36 tiles x 7 splits over 8 XCDs: six XCDs each hold tiles of two K ranges
    {"kernel": "gemm_split_mfma", "plan": "192,320,2,4,2,7", "src": "paper_1309_2734_amd/csrc/gemm.hip",
     "sha": "84eae018c8c7908b", "fetch_kib": 172166.0, "write_kib": 56982.9},
    {"kernel": "direct_fp32", "plan": "8", "src": "paper_1309_2734_amd/csrc/direct.hip",
     "sha": "a2c8df779d41e487", "fetch_kib": 776157.0, "write_kib": 8100.0},
    {"kernel": "direct_fp32", "plan": "16", "src": "paper_1309_2734_amd/csrc/direct.hip",
     "sha": "a2c8df779d41e487", "fetch_kib": 473997.4, "write_kib": 8100.0},
    # the persistent batch GEMM's two launches (one per frame group) of one
    # 64-frame batch, summed
    {"kernel": "gemm_split_mfma_batch", "plan": "384,192,4,2,2",
     "src": "paper_1309_2734_amd/csrc/gemm.hip", "sha": "84eae018c8c7908b",
     "fetch_kib": 23017475.7, "write_kib": 518476.4},
    # the kernels of one diffraction, summed (n = 1024: two column passes;
    # n = 8192: row pass, transpose, row pass, transpose)
    {"kernel": "fresnel_diffraction", "plan": "1024", "src": "paper_1309_2734_amd/csrc/fresnel.hip",
     "sha": "135fcc6b9fcdd374", "fetch_kib": 8510.2, "write_kib": 16384.0},
    {"kernel": "fresnel_diffraction", "plan": "8192", "src": "paper_1309_2734_amd/csrc/fresnel.hip",
     "sha": "135fcc6b9fcdd374", "fetch_kib": 1065685.7, "write_kib": 2097152.1},
]
TRAFFIC_PLANS = {"gemm_split_mfma": ["384,192,4,2,2,8", "192,384,2,4,2,8",
                                     "192,320,2,4,2,7"],
                 "gemm_split_mfma_batch": ["384,192,4,2,2"],
                 "direct_fp32": ["8", "16"], "fresnel_diffraction": ["1024", "8192"]}

# the paper's wavefront-recording times on its K20 (Table 8; context only)
PAPER_TABLE8_GPU_S = {"1000": 0.029, "10000": 0.030, "100000": 0.035}


def _plan_in_tuned(kernel: str, plan: str, tuned) -> bool:
    if kernel == "fresnel_diffraction":
        return plan == tuned
    if kernel == "gemm_split_mfma_batch":
        bm, bn, wm, wn, st = plan.split(",")
        return bool(tuned and f"bm={bm} bn={bn} waves={wm}x{wn} stages={st} " in tuned)
    if kernel.startswith("direct"):
        # the recorded traffic is that of an unsplit launch
        unsplit = bool(tuned and ("splits=1 " in tuned or "splits=0 " in tuned))
        return unsplit and f"rows={plan} " in tuned
    bm, bn, wm, wn, st, sp = plan.split(",")
    return bool(tuned and f"bm={bm} bn={bn} waves={wm}x{wn} stages={st} splits={sp}" in tuned)


def traffic_bytes(kernel: str, tuned):
    """Measured HBM bytes per launch, or None if the kernel or shape changed."""
    import hashlib
    for t in TRAFFIC:
        if t["kernel"] != kernel or not _plan_in_tuned(kernel, t["plan"], tuned):
            continue
        with open(os.path.join(ROOT, t["src"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha"]:
                return None
        return (t["fetch_kib"] * TRAFFIC_SCALE["fetch"] +
                t["write_kib"] * TRAFFIC_SCALE["write"]) * 1024.0
    return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_clock_mhz(run, sync, seconds: float = 0.5):
    """Shader clock while `run` (one step) repeats for about `seconds`: the
    current level of the driver's pp_dpm_sclk files, sampled every ~2 ms from a
    second thread (the step calls release the interpreter lock).  None where
    the files are not readable."""
    import glob
    import re
    import threading
    files = glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")
    if not files:
        return None
    samples, stop = [], threading.Event()

    def sampler():
        while not stop.is_set():
            best = 0
            for f in files:
                try:
                    with open(f) as fh:
                        txt = fh.read()
                except OSError:
                    continue
                for ln in txt.splitlines():
                    mt = re.search(r"(\d+)\s*mhz\s*\*\s*$", ln.strip(), re.I)
                    if mt:
                        best = max(best, int(mt.group(1)))
            if best:
                samples.append(best)
            time.sleep(0.002)

    th = threading.Thread(target=sampler, daemon=True)
    th.start()
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end:
        for _ in range(20):
            run()
        sync()
    stop.set()
    th.join()
    busy = sorted(v for v in samples if v >= 500)     # idle gaps read ~100 MHz
    if not busy:
        return None
    return {"mean": sum(busy) / len(busy), "median": busy[len(busy) // 2], "min": busy[0],
            "max": busy[-1], "samples": len(busy), "source": "pp_dpm_sclk, sampled every ~2 ms "
            f"while the step repeats for ~{seconds:g} s after its timing"}


def _events(torch, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    return e0, e1


def _mfma_roofline(flops, t_ms, peak, kname, traffic=None):
    ach = flops / (t_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
            "traffic": traffic, "kernel": kname, "kernel_ms": t_ms}


def _oracle_rate(pp, dt, threads, sample):
    return {"value": pp / dt, "unit": "point*pixel/s", "cores": threads, "kind": "oracle",
            "sample": sample}


# ------------------------------------------------------------------ legs
# Each leg measures on the GPU and returns (result dict, check), where
# check() runs the oracle on the host afterwards and adds NRMS and max
# errors to the dict.

def bench_modes(args, torch, cghgen, cgh, modes, rows):
    """The headline workload in every mode: tuned, warmed up, K timed steps
    between two synchronisations; per-kernel times from the library's HIP
    events; the shader clock while the step repeats."""
    c = cghgen.make_config(2)
    W, H, N = c.width, c.height, c.n
    pp = W * H * N
    ctx = cgh.Context(W, H, c.pitch, c.wavelength, device=0)
    ctx.upload_cloud(c)
    out = torch.empty((H, W), dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    results = {}
    for m in modes:
        mode = cgh.MODES[m]
        tuned = None
        if not args.no_tune:
            tuned = ctx.tune(mode, repeats=3, stream=stream)
            log(f"mode {m}: tuned {tuned}")
        log(f"mode {m}: warmup {args.warmup}")
        for _ in range(args.warmup):
            ctx.compute(out, mode, stream)
        torch.cuda.synchronize()
        # timed region: K whole steps between two device-wide synchronisations
        log(f"mode {m}: timing {args.steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0, e1 = _events(torch, stream)
        for _ in range(args.steps):
            ctx.compute(out, mode, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ev_ms = e0.elapsed_time(e1) / args.steps
        # per-kernel durations: HIP events around each launch on the same stream
        ctx.profile(True)
        ctx.profile_reset()
        for _ in range(args.steps):
            ctx.compute(out, mode, stream)
        kern = ctx.profile_read()
        ctx.profile(False)
        ctx.compute(out, mode, stream)
        torch.cuda.synchronize()
        sample = out.cpu().numpy()[rows].astype(np.float64)
        clock = measured_clock_mhz(lambda: ctx.compute(out, mode, stream), torch.cuda.synchronize)
        r = {"ms_per_step": wall_ms, "ms_per_step_events": ev_ms, "pp_per_s": pp / (wall_ms * 1e-3),
             "kernels_ms": {k: v[1] / v[0] for k, v in kern.items()},
             "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kern.items()},
             "dtype": MODE_DTYPE[m], "tuned": tuned, "clock_mhz": clock, "_sample": sample}
        if m in ALU_MODES:
            kname, peak = ALU_MODES[m]
            t = r["kernels_ms"].get(kname)
            if t:
                ach = pp / (t * 1e-3)
                r["roofline"] = {"bound": "alu", "achieved": ach, "peak": peak,
                                 "unit": "point*pixel/s", "frac": ach / peak,
                                 "traffic": traffic_bytes(kname, tuned),
                                 "kernel": kname, "kernel_ms": t}
                if m == "direct_fp32":
                    r["roofline"]["peak_issue"] = PEAK_DIRECT_ISSUE_PPS
                    r["roofline"]["frac_issue"] = ach / PEAK_DIRECT_ISSUE_PPS
        else:
            kname = GEMM_KERNEL[m]
            t = r["kernels_ms"].get(kname)
            if t:
                r["roofline"] = _mfma_roofline(
                    FLOP_PER_PP[m] * pp, t, GEMM_PEAK[m], kname,
                    traffic_bytes(kname, tuned) if m == "split_bf16" else None)
        if r.get("roofline") and clock:
            # the same kernel against the peak scaled to the clock it ran at
            r["roofline"]["frac_at_measured_clock"] = (
                r["roofline"]["frac"] * CLOCK_HZ / (clock["median"] * 1e6))
        log(f"mode {m}: {wall_ms:.4f} ms/step, {r['pp_per_s']:.3e} pp/s, kernels {r['kernels_ms']}, "
            f"clock {clock and round(clock['median'])} MHz")
        results[m] = r
    ctx.close()
    return c, results


def bench_batch(args, torch, cghgen, cgh):
    """The batched workload -- F holograms of 1920 x 1080, RGB wavelengths
    cycled, point counts log-uniform in [1e3, 5e4] -- in the FP16 hi/lo split
    mode: tuned for this frame table (cgh_tune_batch), then one
    graph-captured call replayed on a side stream.  The GEMM roofline is the
    persistent batch kernel's 12 flop per point*pixel over its time."""
    b = cghgen.make_batch(n_frames=args.batch_frames)
    frames = cgh.batch_frames(b)
    pp = b.point_pixels
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    out = torch.empty((len(frames), b.height, b.width), device="cuda:0")
    side = torch.cuda.Stream()
    mode = cgh.SPLIT_FP16
    log(f"batch: {len(frames)} frames, {int(b.counts.sum())} points, {pp:.3e} point*pixels")
    tuned = None if args.no_tune else ctx.tune_batch(frames, out, mode, repeats=2, stream=side)
    log(f"batch: tuned {tuned}")
    for _ in range(2):                      # eager run, then capture
        ctx.batch_compute(frames, out, mode, stream=side)
    side.synchronize()
    reps = max(1, min(args.steps, 5))
    e0, e1 = _events(torch, side)
    for _ in range(reps):
        ctx.batch_compute(frames, out, mode, stream=side)
    e1.record(side)
    side.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # per-kernel times of eager calls (profiling runs the sequence eagerly)
    ctx.profile(True)
    ctx.profile_reset()
    for _ in range(2):
        ctx.batch_compute(frames, out, mode, stream=side)
    kern = ctx.profile_read()
    ctx.profile(False)
    side.synchronize()
    kms = {k: v[1] / 2 for k, v in kern.items()}
    gemm_ms = kms.get("gemm_split_mfma_batch")
    # the shader clock while the batch repeats (a sustained matrix-core load)
    clock = measured_clock_mhz(lambda: ctx.batch_compute(frames, out, mode, stream=side),
                               side.synchronize, seconds=1.0)
    cols, rows = cghgen.strided_pixels(b.width, b.height, 8)
    got = out.cpu().numpy()[:, rows][:, :, cols].astype(np.float64)
    ctx.close()
    del out
    torch.cuda.empty_cache()
    log(f"batch: {ms:.3f} ms per batch, {pp / (ms * 1e-3):.3e} pp/s, kernels/batch {kms}")
    res = {"workload": f"{len(frames)} x 1920x1080, RGB 633/532/473 nm, N_f log-uniform "
                       f"[1e3,5e4] (seeds 400+f), {int(b.counts.sum())} points",
           "mode": "split_fp16", "ms_per_batch": ms, "pp_per_s": pp / (ms * 1e-3),
           "launch": "hipGraph replay", "tuned": tuned, "kernels_ms_per_batch": kms,
           "clock_mhz": clock,
           "roofline": _mfma_roofline(12 * pp, gemm_ms, PEAK_MFMA_FP16_TFLOPS,
                                      "gemm_split_mfma_batch",
                                      traffic_bytes("gemm_split_mfma_batch", tuned))
                       if gemm_ms else None}
    if res["roofline"] and clock:
        res["roofline"]["frac_at_measured_clock"] = (
            res["roofline"]["frac"] * CLOCK_HZ / (clock["median"] * 1e6))

    def check():
        import oracle
        threads = oracle.host_threads()
        t0 = time.perf_counter()
        errs, maxes, num, den = [], [], 0.0, 0.0
        for f, (o, n, lam) in enumerate(frames):
            ref = oracle.fresnel(b.width, b.height, b.pitch, lam, b.x[o:o + n], b.y[o:o + n],
                                 b.z[o:o + n], b.amp[o:o + n], cols=cols, rows=rows,
                                 threads=threads)
            errs.append(oracle.nrms(got[f], ref))
            maxes.append(oracle.max_err(got[f], ref))
            num += float(np.sum((got[f] - ref) ** 2))
            den += float(np.sum(ref * ref))
        dt = time.perf_counter() - t0
        spp = len(rows) * len(cols) * int(b.counts.sum())
        res["nrms"] = float(np.sqrt(num / den))
        res["nrms_per_frame_max"] = float(max(errs))
        res["nrms_per_frame_median"] = float(np.median(errs))
        res["max_err"] = float(max(maxes))
        res["cpu_baseline"] = _oracle_rate(
            spp, dt, threads, f"every 8th row and column ({len(rows)} x {len(cols)}) of all "
                              f"{len(frames)} frames, each frame's own points: {spp:.3e} "
                              f"point*pixels in {dt:.1f} s")
        log(f"batch: nrms {res['nrms']:.3e} (frames max {res['nrms_per_frame_max']:.3e}), "
            f"oracle {dt:.1f} s")
    return res, check


def bench_kinoform(args, torch, cghgen, cgh):
    """The phase-only hologram of Eq. (3) (the paper's timed workload) of the
    same 1920 x 1080, 10k-point cloud -- complex field, then the 8-bit phase
    codes -- in three modes.  The codes on every 16th row are then compared
    with the oracle's FP64 field where the device field's error cannot move
    the phase across a code boundary."""
    c = cghgen.make_config(2)
    W, H, N = c.width, c.height, c.n
    pp = W * H * N
    ctx = cgh.Context(W, H, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    stream = torch.cuda.current_stream()
    codes = torch.empty((H, W), dtype=torch.uint8, device="cuda:0")
    field = torch.empty((2, H, W), device="cuda:0")
    rows = np.arange(0, H, 16)
    res, kept = {}, {}
    for m in ("split_bf16", "separable_fp32", "direct_fp32"):
        mode = cgh.MODES[m]
        for _ in range(2):
            ctx.kinoform(codes, mode, stream)
        torch.cuda.synchronize()
        reps = max(1, args.steps)
        e0, e1 = _events(torch, stream)
        for _ in range(reps):
            ctx.kinoform(codes, mode, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        ctx.compute_complex(field, mode, stream)
        torch.cuda.synchronize()
        kept[m] = (field.cpu().numpy().astype(np.float64)[:, rows], codes.cpu().numpy()[rows])
        res[m] = {"ms_per_hologram": ms, "pp_per_s": pp / (ms * 1e-3)}
        log(f"kinoform {m}: {ms:.4f} ms, {res[m]['pp_per_s']:.3e} pp/s")
    ctx.close()
    out = {"workload": "phase-only hologram (Eq. 3) of the 1920x1080, 10000-point cloud: "
                       "complex field + 8-bit phase codes", "modes": res,
           "check": "codes on every 16th row vs the FP64 oracle field, where the device "
                    "field's error cannot cross a code boundary"}

    def check():
        import oracle
        t0 = time.perf_counter()
        ref = oracle.fresnel_complex(W, H, c.pitch, c.wavelength, c.x, c.y, c.z, c.amp,
                                     rows=rows, threads=oracle.host_threads())
        dt = time.perf_counter() - t0
        spp = len(rows) * W * N
        out["cpu_baseline"] = _oracle_rate(
            spp, dt, oracle.host_threads(),
            f"complex field (Eq. (2)) of every 16th row ({len(rows)} rows x {W} columns), all "
            f"{N} points: {spp:.3e} point*pixels in {dt:.1f} s; codes taken from it in FP32")
        t = np.arctan2(ref[1], ref[0])
        t = np.where(t < 0, t + 2 * np.pi, t) * 255.0 / (2 * np.pi)
        mag = np.hypot(ref[0], ref[1])
        want = oracle.kinoform(ref[0], ref[1])
        for m, (f, got) in kept.items():
            e = float(np.max(np.hypot(f[0] - ref[0], f[1] - ref[1])))
            ratio = np.where(mag > 0, e / np.maximum(mag, 1e-300), np.inf)
            margin = np.where(ratio < 0.5, 2 * np.arcsin(np.minimum(ratio, 0.5)) * 255 / (2 * np.pi),
                              np.inf) + 1e-3
            sure = np.abs(t - np.round(t)) > margin
            res[m]["codes_checked"] = int(np.sum(sure))
            res[m]["codes_differing"] = int(np.sum(got[sure] != want[sure]))
            res[m]["codes_differing_any"] = int(np.sum(got != want))
            log(f"kinoform {m}: {res[m]}")
    return out, check


LARGE_MODES = ("split_bf16", "separable_fp32", "direct_fp32")


def _large_set(c, cfg: int):
    """The workload's evaluation set: every 8th row and column of the 2048^2
    cloud; the centred 256 x 256 crop (rows and columns 1920 .. 2175) of the
    4096^2 one."""
    import cghgen
    if cfg == 5:
        return cghgen.crop_pixels(1920, 1920, 256, 256)
    return cghgen.strided_pixels(c.width, c.height, 8)


def bench_large(args, torch, cghgen, cgh):
    """The two large clouds -- 2048 x 2048 with 65,536 points (8 um, 532 nm)
    and 4096 x 4096 with 10^6 points on an ellipsoid surface (4 um; evaluated
    in point chunks that fit the 16 GiB workspace) -- in split BF16, FP32
    separable and direct FP32, each tuned first.  One step = one cgh_compute
    of the whole cloud; the GEMM (or direct) kernel's time is the sum of its
    launches per step.  NRMS and max error against the FP64 oracle on each
    workload's evaluation set."""
    res = {}
    for cfg in (3, 5):
        c = cghgen.make_config(cfg)
        W, H, N = c.width, c.height, c.n
        pp = W * H * N
        steps = 3 if cfg == 3 else 1
        ctx = cgh.Context(W, H, c.pitch, c.wavelength, device=0)
        ctx.upload_cloud(c)
        out = torch.empty((H, W), dtype=torch.float32, device="cuda:0")
        stream = torch.cuda.current_stream()
        cols, rows = _large_set(c, cfg)
        modes = {}
        for m in LARGE_MODES:
            mode = cgh.MODES[m]
            tuned = ctx.tune(mode, repeats=2, stream=stream) if not args.no_tune else None
            ctx.compute(out, mode, stream)               # warm-up
            torch.cuda.synchronize()
            ctx.profile(True)
            ctx.profile_reset()
            e0, e1 = _events(torch, stream)
            for _ in range(steps):
                ctx.compute(out, mode, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            kern = ctx.profile_read()
            ctx.profile(False)
            ms = e0.elapsed_time(e1) / steps
            r = {"ms_per_step": ms, "pp_per_s": pp / (ms * 1e-3), "tuned": tuned,
                 "kernels_ms_per_step": {k: v[1] / steps for k, v in kern.items()},
                 "_got": out.cpu().numpy()[np.ix_(rows, cols)].astype(np.float64)}
            if m in ALU_MODES:
                kname, peak = ALU_MODES[m]
                t = r["kernels_ms_per_step"].get(kname)
                if t:
                    ach = pp / (t * 1e-3)
                    r["roofline"] = {"bound": "alu", "achieved": ach, "peak": peak,
                                     "unit": "point*pixel/s", "frac": ach / peak,
                                     "peak_issue": PEAK_DIRECT_ISSUE_PPS,
                                     "frac_issue": ach / PEAK_DIRECT_ISSUE_PPS,
                                     "kernel": kname, "kernel_ms": t}
            else:
                kname = GEMM_KERNEL[m]
                t = r["kernels_ms_per_step"].get(kname)
                if t:
                    r["roofline"] = _mfma_roofline(FLOP_PER_PP[m] * pp, t, GEMM_PEAK[m], kname)
            log(f"large C{cfg} {m}: {ms:.3f} ms/step, {r['pp_per_s']:.3e} pp/s, "
                f"frac {r.get('roofline', {}).get('frac')}")
            modes[m] = r
        ctx.close()
        del out
        torch.cuda.empty_cache()
        res[f"{W}x{H}_{N}"] = {
            "workload": (f"{W}x{H} hologram, {N} points, pitch {c.pitch * 1e6:g} um, "
                         f"{c.wavelength * 1e9:g} nm (seed {cfg})"),
            "point_pixels_per_step": pp, "steps": steps,
            "evaluation_set": ("every 8th row and column (256 x 256)" if cfg == 3 else
                               "centred 256 x 256 crop, rows and columns 1920..2175"),
            "modes": modes, "_cloud": c, "_set": (cols, rows)}

    def check():
        import oracle
        threads = oracle.host_threads()
        for key, e in res.items():
            c = e.pop("_cloud")
            cols, rows = e.pop("_set")
            t0 = time.perf_counter()
            ref = oracle.cloud_fresnel(c, cols=cols, rows=rows, threads=threads)
            dt = time.perf_counter() - t0
            spp = len(rows) * len(cols) * c.n
            e["cpu_oracle"] = _oracle_rate(spp, dt, threads,
                                           f"{e['evaluation_set']}, all {c.n} points: "
                                           f"{spp:.3e} point*pixels in {dt:.1f} s")
            for m, r in e["modes"].items():
                got = r.pop("_got")
                r["nrms"] = oracle.nrms(got, ref)
                r["max_err"] = oracle.max_err(got, ref)
                log(f"large {key} {m}: nrms {r['nrms']:.3e} max {r['max_err']:.3e}")
    return res, check


SMALL_MODES = ("direct_fp32", "split_bf16", "separable_fp32")


def bench_small(args, torch, cghgen, cgh):
    """The small cloud of the plain method -- 256 x 256, 128 points (8 um,
    632.8 nm) -- in direct FP32 (the form it is specified for) and, beside
    it, split BF16 and FP32 separable: 3 warm-ups, then 20 steps each timed
    with HIP events (median and mean).  A launch of this size is bound by
    launch latency, not by the kernels' arithmetic.  NRMS and max error
    against the FP64 oracle on the full grid."""
    c = cghgen.make_config(1)
    W, H, N = c.width, c.height, c.n
    pp = W * H * N
    ctx = cgh.Context(W, H, c.pitch, c.wavelength, device=0)
    ctx.upload_cloud(c)
    out = torch.empty((H, W), dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    modes = {}
    for m in SMALL_MODES:
        mode = cgh.MODES[m]
        for _ in range(3):
            ctx.compute(out, mode, stream)
        torch.cuda.synchronize()
        times = []
        for _ in range(20):
            e0, e1 = _events(torch, stream)
            ctx.compute(out, mode, stream)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        med = float(np.median(times))
        modes[m] = {"ms_per_step_median": med, "ms_per_step_mean": float(np.mean(times)),
                    "pp_per_s": pp / (med * 1e-3),
                    "_got": out.cpu().numpy().astype(np.float64)}
        log(f"small {m}: {med:.4f} ms/step (median of 20), {pp / (med * 1e-3):.3e} pp/s")
    ctx.close()
    res = {f"{W}x{H}_{N}": {
        "workload": (f"{W}x{H} hologram, {N} points, pitch {c.pitch * 1e6:g} um, "
                     f"{c.wavelength * 1e9:g} nm, x,y ~ U(+-1 mm), z ~ U[0.1,0.2] m, "
                     f"A ~ U[0,1] (seed 1)"),
        "point_pixels_per_step": pp, "evaluation_set": "the full grid", "modes": modes,
        "_cloud": c}}

    def check():
        import oracle
        threads = oracle.host_threads()
        for key, e in res.items():
            cl = e.pop("_cloud")
            t0 = time.perf_counter()
            ref = oracle.cloud_fresnel(cl, threads=threads)
            dt = time.perf_counter() - t0
            e["cpu_oracle"] = _oracle_rate(pp, dt, threads,
                                           f"the full {W}x{H} grid, all {N} points: "
                                           f"{pp:.3e} point*pixels in {dt:.3f} s")
            for m, r in e["modes"].items():
                got = r.pop("_got")
                r["nrms"] = oracle.nrms(got, ref)
                r["max_err"] = oracle.max_err(got, ref)
                log(f"small {key} {m}: nrms {r['nrms']:.3e} max {r['max_err']:.3e}")
    return res, check


def bench_wrm(args, torch, cghgen, cgh):
    """The wavefront-recording method (Section 2.3, Table 8's conditions:
    1920 x 1080 hologram, 8 um, 10^3 .. 10^5 points): per call, the recording
    on the 2048 x 2048 virtual plane 5 mm in front of the shallow object
    (step 1), its Fresnel diffraction to the hologram (step 2) and Re O over
    the hologram window.  NRMS of the recorded plane against the oracle's
    step 1 on sampled rows."""
    zw, n = cghgen.WRM_PLANE_Z, cghgen.WRM_PLANE_N
    res, kept = {}, {}
    stream = torch.cuda.current_stream()
    for npts in (1000, 10000, 100000):
        c = cghgen.make_wrm(npts)
        ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
        ctx.upload_cloud(c)
        plan = cgh.FresnelPlan(n, c.pitch, c.wavelength, zw)
        field = torch.empty((n, n), dtype=torch.complex64, device="cuda:0")
        out = torch.empty((c.height, c.width), device="cuda:0")
        for _ in range(2):
            ctx.wrm_compute(plan, field, out, stream)
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 10))
        e0, e1 = _events(torch, stream)
        for _ in range(reps):
            ctx.wrm_compute(plan, field, out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        ctx.profile(True)
        ctx.profile_reset()
        for _ in range(reps):
            ctx.wrm_compute(plan, field, out, stream)
        kern = ctx.profile_read()
        ctx.profile(False)
        ctx.wrm_record(zw, field, stream)
        torch.cuda.synchronize()
        step = 37 if npts < 100000 else 113
        rows = np.arange(5, n, step)
        kept[npts] = (c, rows, field.cpu().numpy()[rows].astype(np.complex128))
        # point*sample pairs inside the discs: sum of pi r_j^2 / p^2
        d = c.z.astype(np.float64) - zw
        rad = c.wavelength * d / (2 * c.pitch) / c.pitch
        pairs = float(np.sum(np.pi * rad * rad))
        kms = {k: v[1] / v[0] for k, v in kern.items()}
        rec = kms.get("wrm_record")
        rate = pairs / (rec * 1e-3) if rec else None
        r = {"ms_per_hologram": ms, "kernels_ms": kms, "disc_pairs": pairs,
             "record_pairs_per_s": rate,
             "roofline": {"bound": "alu", "achieved": rate, "peak": PEAK_WRM_PAIRS,
                          "unit": "point*sample/s", "frac": rate / PEAK_WRM_PAIRS if rate else None,
                          "traffic": None, "kernel": "wrm_record",
                          "note": "achieved = point*sample pairs inside the discs over the "
                                  "recording kernel's time (chunk planes and their sum "
                                  "included); peak = 8 VALU issue slots per pair (FP64 disc "
                                  "test, selects, complex multiply-add); each wave visits its "
                                  "16x16 sub-tile for every disc that reaches it, ~1.7x the "
                                  "pairs inside the discs at 10^5 points"},
             "paper_table8_gpu_ms": PAPER_TABLE8_GPU_S[str(npts)] * 1e3}
        log(f"wrm N={npts}: {ms:.3f} ms per hologram, kernels {kms}")
        res[str(npts)] = r
        plan.close()
        ctx.close()
        del field, out
    out_res = {"workload": "wavefront-recording method: 1920x1080 hologram, 8 um, 532 nm, "
                           "x,y ~ U(+-3 mm), z ~ U[0.5,0.505] m, A ~ U[0,1] (seed 7); virtual "
                           f"plane {n}x{n} at {zw} m from the hologram (discs 21..42 samples)",
               "points": res, "paper_hardware": "NVIDIA Tesla K20 (Table 8, context only)"}

    def check():
        import oracle
        threads = oracle.host_threads()
        for npts, (c, rows, got) in kept.items():
            t0 = time.perf_counter()
            ref = oracle.wrm_record(n, c.pitch, c.wavelength, zw, c.x, c.y, c.z, c.amp, rows=rows,
                                    threads=threads)
            dt = time.perf_counter() - t0
            e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            res[str(npts)]["record_nrms"] = e
            res[str(npts)]["record_cpu_oracle"] = _oracle_rate(
                len(rows) * n * npts, dt, threads,
                f"recorded plane, {len(rows)} rows x {n} samples, all {npts} points (plain loop, "
                f"no culling) in {dt:.1f} s")
            log(f"wrm N={npts}: record nrms {e:.3e}")
    return out_res, check


def bench_fresnel(args, torch, cgh):
    """Fresnel diffraction of a sampled n x n field (Eq. (10), the second step
    of the wavefront-recording method) at the paper's plane sizes (Table 7:
    n = 1024 .. 8192), random complex fields, z = 0.05 m, 8 um, 532 nm.
    Reports ms per diffraction, the roofline against the algorithm's floor
    (read u, write O: 2 n^2 complex values), the rate of the pipeline's own
    traffic (n <= 1024: 4 n^2 complex values, column convolutions and row
    convolutions read as columns; larger n: 8 n^2, row convolutions,
    transpose, column convolutions, transpose) and the transforms' arithmetic
    rate; the NRMS of n = 1024 against the oracle's FP64 Fourier form."""
    p, lam, z = 8e-6, 532e-9, 0.05
    res, kept = {}, None
    for n in (1024, 2048, 4096, 8192):
        g = torch.Generator(device="cuda:0").manual_seed(n)
        u = torch.randn((n, n), dtype=torch.complex64, device="cuda:0", generator=g)
        out = torch.empty_like(u)
        plan = cgh.FresnelPlan(n, p, lam, z)
        stream = torch.cuda.current_stream()
        for _ in range(2):
            plan.run(u, out, stream)
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 10))
        e0, e1 = _events(torch, stream)
        for _ in range(reps):
            plan.run(u, out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        floor = 2.0 * n * n * 8 / (ms * 1e-3) / 1e9
        planes = 4.0 if n <= 1024 else 8.0
        pipe = planes * n * n * 8 / (ms * 1e-3) / 1e9
        # 2n line convolutions of length L = 2n: two transforms (5 L log2 L
        # flop each, the radix-2 count) and the spectrum product (6 L)
        L = 2 * n
        flop = 2.0 * n * (2 * 5.0 * L * math.log2(L) + 6.0 * L)
        tf = flop / (ms * 1e-3) / 1e12
        r = {"ms": ms, "pipeline_gb_per_s": pipe, "pipeline_frac": pipe / PEAK_HBM_GBS,
             "roofline": {"bound": "hbm", "achieved": floor, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": floor / PEAK_HBM_GBS,
                          "traffic": traffic_bytes("fresnel_diffraction", str(n)),
                          "note": "achieved = the algorithm's floor, 2 n^2 x 8 B (read u, write "
                                  f"O), over the whole diffraction time; the pipeline moves "
                                  f"{planes / 2:.0f}x that (pipeline_gb_per_s); traffic = "
                                  "counter-measured HBM bytes of one diffraction (recorded for "
                                  "n = 1024 and 8192)"},
             "alu": {"achieved": tf, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf / PEAK_FP32_VALU_TFLOPS,
                     "note": "the transforms' arithmetic, 2n lines x (2 x 5 L log2 L + 6 L) "
                             "flop, L = 2n, over the whole diffraction time, against FP32 "
                             "vector multiply-adds without packed operations (256 CUs x 64 "
                             "lanes x 2 flop x 2.4 GHz)"}}
        if n == 1024:
            kept = (u.cpu().numpy().astype(np.complex128), out.cpu().numpy().astype(np.complex128))
        plan.close()
        log(f"fresnel n={n}: {ms:.3f} ms")
        res[str(n)] = r
    out_res = {"workload": "Fresnel diffraction (Eq. 10) of a random complex n x n field, "
                           "zero-padded FFTs on the 2n grid, 8 um, 532 nm, z = 0.05 m",
               "n": res,
               "paper_table7_gpu_s": {"1024": 0.011, "2048": 0.027, "4096": 0.125, "8192": None},
               "paper_hardware": "NVIDIA Tesla K20, CUFFT (context only)"}

    def check():
        import oracle
        uh, got = kept
        t0 = time.perf_counter()
        ref = oracle.diffraction_fft(uh, p, lam, z)
        cpu_s = time.perf_counter() - t0
        r = res["1024"]
        r["nrms"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        r["cpu_baseline"] = {"value": cpu_s * 1e3, "unit": "ms per diffraction", "cores": 1,
                             "kind": "oracle",
                             "sample": "the whole n = 1024 diffraction, FP64 Fourier form "
                                       "(numpy FFTs, one thread)"}
        log(f"fresnel n=1024: nrms {r['nrms']:.3e}")
    return out_res, check


def bench_vendor_gemm(args, torch, kblocks_points: int):
    """Context, not the path: the vendor BLAS (torch.matmul, hipBLASLt) on a
    plain BF16 GEMM of the split GEMM's flop count at 1920x1080 -- the three
    products as one product over K = 3 x 2 x (points padded), both operands
    contiguous -- so the matrix-core fraction of the hand-written kernel can
    be read against the library's on the same shape."""
    M, N, K = 1080, 1920, 3 * 2 * kblocks_points
    g = torch.Generator(device="cuda:0").manual_seed(11)
    a = torch.randn((M, K), dtype=torch.bfloat16, device="cuda:0", generator=g)
    b = torch.randn((K, N), dtype=torch.bfloat16, device="cuda:0", generator=g)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        c = torch.matmul(a, b)
    torch.cuda.synchronize()
    reps = 10
    e0, e1 = _events(torch, stream)
    for _ in range(reps):
        c = torch.matmul(a, b)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tf = 2.0 * M * N * K / (ms * 1e-3) / 1e12
    del a, b, c
    log(f"vendor GEMM {M}x{N}x{K}: {ms:.3f} ms, {tf:.0f} TFLOP/s")
    return {"shape": [M, N, K], "ms": ms, "tflops": tf, "frac": tf / PEAK_MFMA_BF16_TFLOPS,
            "note": "context only: torch.matmul (hipBLASLt), BF16 in and out, FP32 "
                    "accumulation, on the split GEMM's flop count; not part of the path"}


def traffic_driver(torch, cghgen, cgh) -> int:
    """Kernel sequence for `rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE -- python bench.py
    --traffic-driver`: the per-launch counters of the split-BF16 GEMM in each recorded
    launch shape (3 computes each), of the one-product FP16 GEMM in the first of them
    (2 computes), of the direct kernel at each recorded row count
    (2 computes each), of the four kernels of a Fresnel diffraction at each recorded
    size (2 runs), of the exact spherical wave (2 computes, unsplit), of the
    wavefront recording of 10^5 points (2 runs), of the 64-frame
    batch's persistent GEMM in each recorded shape (one eager batch: one launch per
    frame group), and of a plain 256 MiB device copy (3 copies) whose true byte counts
    calibrate them.  Tuned plans are not read (a tuned plan would take precedence over
    the launch shapes set here)."""
    os.environ.pop("CGH_TUNE_CACHE", None)
    c = cghgen.make_config(2)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    out = torch.empty((c.height, c.width), device="cuda:0")
    for plan in TRAFFIC_PLANS["gemm_split_mfma"]:
        os.environ["CGH_GEMM_PLAN"] = plan
        for _ in range(3):
            ctx.compute(out, cgh.SPLIT_BF16)
        torch.cuda.synchronize()
        log(f"traffic driver: split_bf16 plan {plan}")
    os.environ["CGH_GEMM_PLAN"] = TRAFFIC_PLANS["gemm_split_mfma"][0]
    for _ in range(2):                              # one product, FP16, the same shape
        ctx.compute(out, cgh.FP16)
    torch.cuda.synchronize()
    log("traffic driver: fp16")
    os.environ.pop("CGH_GEMM_PLAN", None)
    os.environ["CGH_DIRECT_SPLITS"] = "1"           # the recorded launches are unsplit
    for rows in TRAFFIC_PLANS["direct_fp32"]:
        os.environ["CGH_DIRECT_ROWS"] = rows
        for _ in range(2):
            ctx.compute(out, cgh.DIRECT_FP32)
        torch.cuda.synchronize()
        log(f"traffic driver: direct rows {rows}")
    os.environ.pop("CGH_DIRECT_ROWS", None)
    for _ in range(2):                              # the exact spherical wave, default shape
        ctx.compute(out, cgh.SPHERICAL_FP32)
    torch.cuda.synchronize()
    log("traffic driver: spherical")
    os.environ.pop("CGH_DIRECT_SPLITS", None)
    for n in TRAFFIC_PLANS["fresnel_diffraction"]:
        g = torch.Generator(device="cuda:0").manual_seed(int(n))
        u = torch.randn((int(n), int(n)), dtype=torch.complex64, device="cuda:0", generator=g)
        o = torch.empty_like(u)
        plan = cgh.FresnelPlan(int(n), 8e-6, 532e-9, 0.05)
        for _ in range(2):
            plan.run(u, o)
        torch.cuda.synchronize()
        plan.close()
        del u, o
        log(f"traffic driver: Fresnel diffraction n={n}")
    w = cghgen.make_wrm(100000)
    wctx = cgh.Context(w.width, w.height, w.pitch, w.wavelength)
    wctx.upload_cloud(w)
    field = torch.empty((cghgen.WRM_PLANE_N, cghgen.WRM_PLANE_N), dtype=torch.complex64,
                        device="cuda:0")
    for _ in range(2):
        wctx.wrm_record(cghgen.WRM_PLANE_Z, field)
    torch.cuda.synchronize()
    wctx.close()
    del field
    log("traffic driver: wavefront recording, 1e5 points")
    b = cghgen.make_batch(64)
    frames = cgh.batch_frames(b)
    bctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    bctx.upload_cloud(b)
    bout = torch.empty((len(frames), b.height, b.width), device="cuda:0")
    bctx.profile(True)                      # profiled calls run eagerly (no graph)
    for plan in TRAFFIC_PLANS["gemm_split_mfma_batch"]:
        os.environ["CGH_GEMM_PLAN"] = plan
        bctx.batch_compute(frames, bout, cgh.SPLIT_FP16)
        torch.cuda.synchronize()
        log(f"traffic driver: batch plan {plan}")
    os.environ.pop("CGH_GEMM_PLAN", None)
    bctx.close()
    del bout
    src = torch.ones(64 << 20, device="cuda:0")       # 256 MiB of float32
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    log("traffic driver done")
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default="split_bf16,direct_fp32,separable_fp32,split_fp16,fp16,"
                                       "spherical_fp32",
                    help="comma list; the first is the headline mode")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (profiling runs)")
    ap.add_argument("--sample-row-step", type=int, default=3)
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shapes")
    ap.add_argument("--no-kinoform", action="store_true",
                    help="skip the phase-only hologram side measurement")
    ap.add_argument("--no-fresnel", action="store_true",
                    help="skip the Fresnel-diffraction side measurement")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2048x2048 / 4096x4096 side measurement")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 256x256, 128-point side measurement")
    ap.add_argument("--no-wrm", action="store_true",
                    help="skip the wavefront-recording side measurement")
    ap.add_argument("--batch-frames", type=int, default=64,
                    help="frames of the batched-workload side measurement (0 = skip)")
    ap.add_argument("--traffic-driver", action="store_true",
                    help="run only the fixed kernel sequence the HBM-traffic counter passes "
                         "read (split-BF16 computes in each recorded GEMM shape, direct "
                         "computes at each recorded row count, 3 device copies of 256 MiB "
                         "for calibration), then exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU per process and this benchmark measures one; "
              "--gpus must be 1", file=sys.stderr)
        return 2

    import torch

    import cghgen
    import paper_1309_2734_amd as cgh

    if args.traffic_driver:
        return traffic_driver(torch, cghgen, cgh)

    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    head = modes[0]
    torch.cuda.set_device(0)
    H = 1080
    rows = np.arange(0, H, args.sample_row_step)

    # ---- GPU phase
    c, results = bench_modes(args, torch, cghgen, cgh, modes, rows)
    W, H, N = c.width, c.height, c.n
    pp = W * H * N
    legs = {}
    if args.batch_frames > 0:
        legs["batch"] = bench_batch(args, torch, cghgen, cgh)
    if not args.no_kinoform:
        legs["kinoform"] = bench_kinoform(args, torch, cghgen, cgh)
    if not args.no_small:
        legs["small"] = bench_small(args, torch, cghgen, cgh)
    if not args.no_large:
        legs["large"] = bench_large(args, torch, cghgen, cgh)
    if not args.no_wrm:
        legs["wrm"] = bench_wrm(args, torch, cghgen, cgh)
    if not args.no_fresnel:
        legs["fresnel_diffraction"] = bench_fresnel(args, torch, cgh)
    vendor = bench_vendor_gemm(args, torch, (c.n + 31) // 32 * 32)

    # ---- host phase: the oracle alone on the host cores
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.host_threads()
        log(f"oracle on {len(rows)} rows x {W} cols x {N} points, {threads} threads")
        t0 = time.perf_counter()
        ref = oracle.cloud_fresnel(c, rows=rows, threads=threads)
        dt = time.perf_counter() - t0
        sample_pp = len(rows) * W * N
        cpu = _oracle_rate(sample_pp, dt, threads,
                           f"every {args.sample_row_step}-th row ({len(rows)} rows x {W} columns) "
                           f"of the {W}x{H} hologram, all {N} points: {sample_pp:.3e} "
                           f"point*pixels in {dt:.1f} s (FP64, libm cos)")
        # the same oracle on one core, on the small 256 x 256, 128-point cloud
        c1 = cghgen.make_config(1)
        t0 = time.perf_counter()
        oracle.cloud_fresnel(c1, threads=1)
        dt1 = time.perf_counter() - t0
        pp1 = c1.width * c1.height * c1.n
        cpu["one_core"] = {"value": pp1 / dt1, "unit": "point*pixel/s", "cores": 1,
                           "sample": f"full {c1.width}x{c1.height} grid, {c1.n} points: "
                                     f"{pp1:.3e} point*pixels in {dt1:.3f} s"}
        log(f"oracle on one core, 256x256 x 128: {pp1 / dt1:.3e} pp/s")
        for m, r in results.items():
            if m == "spherical_fp32":
                # Eq. (1) has its own reference: every 4th sample row
                srows = rows[::4]
                t0 = time.perf_counter()
                sph = oracle.spherical_complex(W, H, c.pitch, c.wavelength, c.x, c.y, c.z, c.amp,
                                               rows=srows, threads=threads)[0]
                dt = time.perf_counter() - t0
                spp = len(srows) * W * N
                r["cpu_baseline"] = _oracle_rate(
                    spp, dt, threads, f"Eq. (1) with its imaginary part, every "
                                      f"{4 * args.sample_row_step}-th row ({len(srows)} rows x "
                                      f"{W} columns), all {N} points: {spp:.3e} point*pixels in "
                                      f"{dt:.1f} s")
                got, want = r["_sample"][::4], sph
            else:
                got, want = r["_sample"], ref
            r["nrms"] = oracle.nrms(got, want)
            r["max_err"] = oracle.max_err(got, want)
            log(f"mode {m}: nrms {r['nrms']:.3e} max {r['max_err']:.3e}")
        for name, (res, check) in legs.items():
            log(f"oracle for {name}")
            check()
    for r in results.values():
        r.pop("_sample", None)
    for name in ("small", "large"):
        if name in legs:
            for e in legs[name][0].values():
                e.pop("_cloud", None)
                e.pop("_set", None)
                for r in e["modes"].values():
                    r.pop("_got", None)

    h = results[head]
    line = {
        "metric": "point*pixel/s at 1920x1080, 10k points (direct FP32 vs MFMA split); NRMS vs FP64",
        "value": h["pp_per_s"],
        "unit": "point*pixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": h["dtype"],
        "data": "synthetic",
        "config": {"workload": "1920x1080 hologram, 10000 points, pitch 8 um, 532 nm, "
                               "x,y ~ U(+-3 mm), z ~ U[0.5,0.6] m, A ~ U[0,1] (seed 2)",
                   "mode": head, "point_pixels_per_step": pp},
        "nrms": h.get("nrms"),
        "max_err": h.get("max_err"),
        "nrms_set": f"every {args.sample_row_step}-th row of the hologram vs the FP64 oracle",
        "roofline": h.get("roofline"),
        "cpu_baseline": cpu,
        # the same workload in FP32 arithmetic (the paper's precision), beside the split
        "fp32": {m: {"value": results[m]["pp_per_s"], "unit": "point*pixel/s",
                     "ms_per_step": results[m]["ms_per_step"],
                     "frac": (results[m].get("roofline") or {}).get("frac"),
                     "nrms": results[m].get("nrms")}
                 for m in ("direct_fp32", "separable_fp32") if m in results},
        "modes": results,
        "vendor_gemm": vendor,
    }
    for name, (res, _) in legs.items():
        line[name] = res
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
