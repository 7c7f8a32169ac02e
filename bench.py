"""Benchmark: point*pixel/s of the hologram hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: a 1920 x 1080 hologram of 10,000 points (8 um pitch, 532 nm,
x, y ~ U(+-3 mm), z ~ U[0.5, 0.6] m, A ~ U[0, 1]; seeded synthetic cloud,
cghgen config 2), points resident in HBM before timing.  One step = one
cgh_compute of the whole cloud in the headline mode (BF16 hi/lo split on the
matrix cores: per-point constants, factor build, split GEMM, split-K reduce).
The direct FP32 kernel and the other modes are timed the same way and
reported under "modes" (spherical_fp32 evaluates the exact spherical wave of
Eq. (1) instead of the Fresnel sum).  NRMS and max error of every mode are
measured against the FP64 oracle on the CPU-baseline sample (every 4th row;
every 16th for the spherical mode, against the oracle's Eq. (1)).  Side
measurements: the 64-frame batched workload ("batch"), the phase-only
hologram of Eq. (3) of the bench cloud ("kinoform"), and the Fresnel
diffraction of Eq. (10) at the paper's plane sizes ("fresnel_diffraction").

Prints one JSON line (rank 0).  --gpus N > 1 is refused: the benchmark
measures one GPU.
"""
from __future__ import annotations

import argparse
import json
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
# exact spherical wave: 2 v_add_f32_dpp, 2 v_add_f32, 2 v_mul_f32, v_fma_f32,
# v_fmac_f32 and v_sqrt_f32, v_rcp_f32, v_cos_f32 per point*pixel
PEAK_SPHERE_PPS = alu_peak_pps(11, 3)         # 3.575e12 point*pixel/s
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
     "sha": "c2a5d793680ad21f", "fetch_kib": 120352.0, "write_kib": 64800.1},
    {"kernel": "gemm_split_mfma", "plan": "192,384,2,4,2,8", "src": "paper_1309_2734_amd/csrc/gemm.hip",
     "sha": "c2a5d793680ad21f", "fetch_kib": 120352.0, "write_kib": 64800.6},
    {"kernel": "direct_fp32", "plan": "8", "src": "paper_1309_2734_amd/csrc/direct.hip",
     "sha": "d5d17ae7d96a2dcc", "fetch_kib": 776234.7, "write_kib": 8100.0},
    {"kernel": "direct_fp32", "plan": "16", "src": "paper_1309_2734_amd/csrc/direct.hip",
     "sha": "d5d17ae7d96a2dcc", "fetch_kib": 474243.2, "write_kib": 8100.0},
    # the five kernels of one n = 8192 diffraction, summed
    {"kernel": "fresnel_diffraction", "plan": "8192", "src": "paper_1309_2734_amd/csrc/fresnel.hip",
     "sha": "901dbb79b87cb5d5", "fetch_kib": 2376938.1, "write_kib": 4718593.0},
]
TRAFFIC_PLANS = {"gemm_split_mfma": ["384,192,4,2,2,8", "192,384,2,4,2,8"],
                 "direct_fp32": ["8", "16"], "fresnel_diffraction": ["8192"]}


def _plan_in_tuned(kernel: str, plan: str, tuned) -> bool:
    if kernel == "fresnel_diffraction":
        return plan == tuned
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
            "while the step repeats for ~0.5 s after its timing"}


def bench_batch(args, torch, cghgen, cgh, check: bool):
    """Side measurement: the batched workload -- F holograms of 1920 x 1080,
    RGB wavelengths cycled, point counts log-uniform in [1e3, 5e4] -- in the
    FP16 hi/lo split mode through one graph-captured launch sequence on a
    side stream.  Reports point*pixel/s over all frames and (with the CPU
    baseline on) the NRMS of two frames against the FP64 oracle on a strided
    sample."""
    b = cghgen.make_batch(n_frames=args.batch_frames)
    frames = cgh.batch_frames(b)
    pp = b.point_pixels
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    out = torch.empty((len(frames), b.height, b.width), device="cuda:0")
    side = torch.cuda.Stream()
    mode = cgh.SPLIT_FP16
    log(f"batch: {len(frames)} frames, {int(b.counts.sum())} points, {pp:.3e} point*pixels")
    for _ in range(2):                      # eager run, then capture
        ctx.batch_compute(frames, out, mode, stream=side)
    side.synchronize()
    reps = max(1, min(args.steps, 5))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(side)
    for _ in range(reps):
        ctx.batch_compute(frames, out, mode, stream=side)
    e1.record(side)
    side.synchronize()
    ms = e0.elapsed_time(e1) / reps
    rows, cols = np.arange(0, b.height, 16), np.arange(0, b.width, 16)
    errs = []
    for f in ((0, len(frames) - 1) if check else ()):
        import oracle
        o, n, lam = frames[f]
        ref = oracle.fresnel(b.width, b.height, b.pitch, lam, b.x[o:o + n], b.y[o:o + n],
                             b.z[o:o + n], b.amp[o:o + n], cols=cols, rows=rows)
        got = out[f].cpu().numpy().astype(np.float64)[np.ix_(rows, cols)]
        errs.append(oracle.nrms(got, ref))
    ctx.close()
    log(f"batch: {ms:.3f} ms per batch, {pp / (ms * 1e-3):.3e} pp/s, nrms {errs}")
    return {"workload": f"{len(frames)} x 1920x1080, RGB 633/532/473 nm, N_f log-uniform "
                        f"[1e3,5e4] (seeds 400+f), {int(b.counts.sum())} points",
            "mode": "split_fp16", "ms_per_batch": ms, "pp_per_s": pp / (ms * 1e-3),
            "launch": "hipGraph replay", "nrms_sampled_frames": errs}


def bench_kinoform(args, torch, cghgen, cgh, check: bool):
    """Side measurement: the phase-only hologram of Eq. (3) (the paper's
    timed workload) of the same 1920 x 1080, 10k-point cloud -- complex
    field, then the 8-bit phase codes -- in three modes.  With `check`, the
    codes on every 16th row are compared with the oracle's FP64 field where
    the device field's error cannot move the phase across a code boundary."""
    c = cghgen.make_config(2)
    W, H, N = c.width, c.height, c.n
    pp = W * H * N
    ctx = cgh.Context(W, H, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    stream = torch.cuda.current_stream()
    codes = torch.empty((H, W), dtype=torch.uint8, device="cuda:0")
    field = torch.empty((2, H, W), device="cuda:0")
    rows = np.arange(0, H, 16)
    ref = None
    cpu = None
    if check:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.fresnel_complex(W, H, c.pitch, c.wavelength, c.x, c.y, c.z, c.amp,
                                     rows=rows, threads=oracle.host_threads())
        dt = time.perf_counter() - t0
        spp = len(rows) * W * N
        cpu = {"value": spp / dt, "unit": "point*pixel/s", "cores": oracle.host_threads(),
               "kind": "oracle",
               "sample": f"complex field (Eq. (2)) of every 16th row ({len(rows)} rows x {W} "
                         f"columns), all {N} points: {spp:.3e} point*pixels in {dt:.1f} s; "
                         f"codes taken from it in FP64"}
    res = {}
    for m in ("split_bf16", "separable_fp32", "direct_fp32"):
        mode = cgh.MODES[m]
        for _ in range(2):
            ctx.kinoform(codes, mode, stream)
        torch.cuda.synchronize()
        reps = max(1, args.steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            ctx.kinoform(codes, mode, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        r = {"ms_per_hologram": ms, "pp_per_s": pp / (ms * 1e-3)}
        if ref is not None:
            ctx.compute_complex(field, mode, stream)
            torch.cuda.synchronize()
            f = field.cpu().numpy().astype(np.float64)[:, rows]
            got = codes.cpu().numpy()[rows]
            import oracle
            t = np.arctan2(ref[1], ref[0])
            t = np.where(t < 0, t + 2 * np.pi, t) * 255.0 / (2 * np.pi)
            mag = np.hypot(ref[0], ref[1])
            e = float(np.max(np.hypot(f[0] - ref[0], f[1] - ref[1])))
            ratio = np.where(mag > 0, e / np.maximum(mag, 1e-300), np.inf)
            margin = np.where(ratio < 0.5, 2 * np.arcsin(np.minimum(ratio, 0.5)) * 255 / (2 * np.pi),
                              np.inf) + 1e-3
            sure = np.abs(t - np.round(t)) > margin
            want = oracle.kinoform(ref[0], ref[1])
            r["codes_checked"] = int(np.sum(sure))
            r["codes_differing"] = int(np.sum(got[sure] != want[sure]))
            r["codes_differing_any"] = int(np.sum(got != want))
        log(f"kinoform {m}: {ms:.4f} ms, {r['pp_per_s']:.3e} pp/s {r}")
        res[m] = r
    ctx.close()
    return {"workload": "phase-only hologram (Eq. 3) of the 1920x1080, 10000-point cloud: "
                        "complex field + 8-bit phase codes", "modes": res,
            "check": "codes on every 16th row vs the FP64 oracle field, where the device "
                     "field's error cannot cross a code boundary" if check else None,
            "cpu_baseline": cpu}


def bench_fresnel(args, torch, cgh, check: bool):
    """Side measurement: Fresnel diffraction of a sampled n x n field (Eq. (10),
    the second step of the wavefront-recording method) at the paper's plane sizes
    (Table 7: n = 1024 .. 8192), random complex fields, z = 0.05 m, 8 um, 532 nm.
    Reports ms per diffraction and the effective HBM rate of the pruned pipeline
    (18 n^2 complex values moved); with `check`, the NRMS of n = 1024 against the
    oracle's FP64 Fourier form."""
    p, lam, z = 8e-6, 532e-9, 0.05
    res = {}
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
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.run(u, out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = 18.0 * n * n * 8 / (ms * 1e-3) / 1e9
        r = {"ms": ms, "hbm_gb_per_s": gbs,
             "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": gbs / PEAK_HBM_GBS,
                          "traffic": traffic_bytes("fresnel_diffraction", str(n)),
                          "note": "achieved = the five-kernel pipeline's 18 n^2 x 8 B over the "
                                  "whole diffraction time; traffic = counter-measured HBM "
                                  "bytes of one diffraction (recorded for n = 8192)"}}
        if check and n == 1024:
            import oracle
            uh = u.cpu().numpy().astype(np.complex128)
            t0 = time.perf_counter()
            ref = oracle.diffraction_fft(uh, p, lam, z)
            cpu_s = time.perf_counter() - t0
            got = out.cpu().numpy().astype(np.complex128)
            r["nrms"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            r["cpu_baseline"] = {"value": cpu_s * 1e3, "unit": "ms per diffraction", "cores": 1,
                                 "kind": "oracle",
                                 "sample": "the whole n = 1024 diffraction, FP64 Fourier form "
                                           "(numpy FFTs, one thread)"}
        plan.close()
        log(f"fresnel n={n}: {ms:.3f} ms {r}")
        res[str(n)] = r
    return {"workload": "Fresnel diffraction (Eq. 10) of a random complex n x n field, "
                        "zero-padded FFTs on the 2n grid, 8 um, 532 nm, z = 0.05 m",
            "n": res,
            "paper_table7_gpu_s": {"1024": 0.011, "2048": 0.027, "4096": 0.125, "8192": None},
            "paper_hardware": "NVIDIA Tesla K20, CUFFT (context only)"}


LARGE_MODES = ("split_bf16", "separable_fp32", "direct_fp32")


def _large_sample(c, cfg: int):
    """The strided pixel sample the parity tests use at these sizes."""
    if cfg == 5:
        return np.arange(7, c.width, 160), np.arange(3, c.height, 160)
    cols = np.array(sorted(set(range(0, c.width, 64)) | {c.width - 1}))
    rows = np.array(sorted(set(range(0, c.height, 64)) | {c.height - 1}))
    return cols, rows


def bench_large(args, torch, cghgen, cgh, check: bool):
    """Side measurement: the two large clouds -- 2048 x 2048 with 65,536
    points (8 um, 532 nm) and 4096 x 4096 with 10^6 points on an ellipsoid
    surface (4 um; evaluated in point chunks that fit the 16 GiB workspace)
    -- in split BF16, FP32 separable and direct FP32, each tuned first.  One
    step = one cgh_compute of the whole cloud; the GEMM (or direct) kernel's
    time is the sum of its launches per step.  With the CPU baseline on,
    NRMS and max error against the FP64 oracle on the strided sample the
    parity tests use."""
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
        cols, rows = _large_sample(c, cfg)
        ref = None
        oracle_rate = None
        if check:
            import oracle
            threads = oracle.host_threads()
            t0 = time.perf_counter()
            ref = oracle.cloud_fresnel(c, cols=cols, rows=rows, threads=threads)
            dt = time.perf_counter() - t0
            spp = len(rows) * len(cols) * N
            oracle_rate = {"value": spp / dt, "unit": "point*pixel/s", "cores": threads,
                           "kind": "oracle", "sample": f"{len(rows)} x {len(cols)} strided pixels, "
                                                       f"all {N} points: {spp:.3e} point*pixels "
                                                       f"in {dt:.2f} s"}
            log(f"large C{cfg}: oracle sample {len(rows)}x{len(cols)} in {dt:.1f} s")
        modes = {}
        for m in LARGE_MODES:
            mode = cgh.MODES[m]
            tuned = ctx.tune(mode, repeats=2, stream=stream) if not args.no_tune else None
            ctx.compute(out, mode, stream)               # warm-up
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            ctx.profile(True)
            ctx.profile_reset()
            e0.record(stream)
            for _ in range(steps):
                ctx.compute(out, mode, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            kern = ctx.profile_read()
            ctx.profile(False)
            ms = e0.elapsed_time(e1) / steps
            r = {"ms_per_step": ms, "pp_per_s": pp / (ms * 1e-3), "tuned": tuned,
                 "kernels_ms_per_step": {k: v[1] / steps for k, v in kern.items()}}
            if m in ALU_MODES:
                kname, peak = ALU_MODES[m]
                t = r["kernels_ms_per_step"].get(kname)
                if t:
                    ach = pp / (t * 1e-3)
                    r["roofline"] = {"bound": "alu", "achieved": ach, "peak": peak,
                                     "unit": "point*pixel/s", "frac": ach / peak,
                                     "kernel": kname, "kernel_ms": t}
            else:
                kname = GEMM_KERNEL[m]
                t = r["kernels_ms_per_step"].get(kname)
                if t:
                    ach = FLOP_PER_PP[m] * pp / (t * 1e-3) / 1e12
                    r["roofline"] = {"bound": "mfma", "achieved": ach, "peak": GEMM_PEAK[m],
                                     "unit": "TFLOP/s", "frac": ach / GEMM_PEAK[m],
                                     "kernel": kname, "kernel_ms": t}
            if ref is not None:
                import oracle
                got = out.cpu().numpy()[np.ix_(rows, cols)].astype(np.float64)
                r["nrms"] = oracle.nrms(got, ref)
                r["max_err"] = oracle.max_err(got, ref)
            log(f"large C{cfg} {m}: {ms:.3f} ms/step, {r['pp_per_s']:.3e} pp/s, "
                f"frac {r.get('roofline', {}).get('frac')}, nrms {r.get('nrms')}")
            modes[m] = r
        ctx.close()
        del out
        torch.cuda.empty_cache()
        res[f"{W}x{H}_{N}"] = {
            "workload": (f"{W}x{H} hologram, {N} points, pitch {c.pitch * 1e6:g} um, "
                         f"{c.wavelength * 1e9:g} nm (seed {cfg})"),
            "point_pixels_per_step": pp, "steps": steps,
            "sample": f"{len(rows)} rows x {len(cols)} columns, strided" if check else None,
            "cpu_oracle": oracle_rate, "modes": modes}
    return res


def traffic_driver(torch, cghgen, cgh) -> int:
    """Kernel sequence for `rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE -- python bench.py
    --traffic-driver`: the per-launch counters of the split-BF16 GEMM in each recorded
    launch shape (3 computes each), of the direct kernel at each recorded row count
    (2 computes each), of the five kernels of a Fresnel diffraction at each recorded
    size (2 runs), and of a plain 256 MiB device copy (3 copies) whose true byte
    counts calibrate them."""
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
    os.environ.pop("CGH_GEMM_PLAN", None)
    os.environ["CGH_DIRECT_SPLITS"] = "1"           # the recorded launches are unsplit
    for rows in TRAFFIC_PLANS["direct_fp32"]:
        os.environ["CGH_DIRECT_ROWS"] = rows
        for _ in range(2):
            ctx.compute(out, cgh.DIRECT_FP32)
        torch.cuda.synchronize()
        log(f"traffic driver: direct rows {rows}")
    os.environ.pop("CGH_DIRECT_ROWS", None)
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
    ap.add_argument("--sample-row-step", type=int, default=4)
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shapes")
    ap.add_argument("--no-kinoform", action="store_true",
                    help="skip the phase-only hologram side measurement")
    ap.add_argument("--no-fresnel", action="store_true",
                    help="skip the Fresnel-diffraction side measurement")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2048x2048 / 4096x4096 side measurement")
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
    c = cghgen.make_config(2)
    W, H, N = c.width, c.height, c.n
    pp = W * H * N
    ctx = cgh.Context(W, H, c.pitch, c.wavelength, device=0)
    ctx.upload_cloud(c)
    out = torch.empty((H, W), dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    rows = np.arange(0, H, args.sample_row_step)

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
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
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
             "kernels_ms": {k: v[1] / v[0] for k, v in kern.items()}, "sample": sample,
             "dtype": MODE_DTYPE[m], "tuned": tuned, "clock_mhz": clock}
        if m in ALU_MODES:
            kname, peak = ALU_MODES[m]
            t = r["kernels_ms"].get(kname)
            if t:
                ach = pp / (t * 1e-3)
                r["roofline"] = {"bound": "alu", "achieved": ach, "peak": peak,
                                 "unit": "point*pixel/s", "frac": ach / peak,
                                 "traffic": traffic_bytes(kname, tuned),
                                 "kernel": kname, "kernel_ms": t}
        else:
            kname = GEMM_KERNEL[m]
            t = r["kernels_ms"].get(kname)
            if t:
                flops = FLOP_PER_PP[m] * pp
                ach = flops / (t * 1e-3) / 1e12
                peak = GEMM_PEAK[m]
                r["roofline"] = {"bound": "mfma", "achieved": ach, "peak": peak,
                                 "unit": "TFLOP/s", "frac": ach / peak,
                                 "traffic": traffic_bytes(kname, tuned) if m == "split_bf16"
                                 else None, "kernel": kname, "kernel_ms": t}
        if r.get("roofline") and clock:
            # the same kernel against the peak scaled to the clock it ran at
            r["roofline"]["frac_at_measured_clock"] = (
                r["roofline"]["frac"] * CLOCK_HZ / (clock["median"] * 1e6))
        log(f"mode {m}: {wall_ms:.4f} ms/step, {r['pp_per_s']:.3e} pp/s, kernels {r['kernels_ms']}, "
            f"clock {clock and round(clock['median'])} MHz")
        results[m] = r
    ctx.close()

    batch = None
    if args.batch_frames > 0:
        batch = bench_batch(args, torch, cghgen, cgh, check=not args.no_cpu_baseline)
    kino = None
    if not args.no_kinoform:
        kino = bench_kinoform(args, torch, cghgen, cgh, check=not args.no_cpu_baseline)
    large = None
    if not args.no_large:
        large = bench_large(args, torch, cghgen, cgh, check=not args.no_cpu_baseline)
    fres = None
    if not args.no_fresnel:
        fres = bench_fresnel(args, torch, cgh, check=not args.no_cpu_baseline)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.host_threads()
        log(f"oracle on {len(rows)} rows x {W} cols x {N} points, {threads} threads")
        t0 = time.perf_counter()
        ref = oracle.cloud_fresnel(c, rows=rows, threads=threads)
        dt = time.perf_counter() - t0
        sample_pp = len(rows) * W * N
        cpu = {"value": sample_pp / dt, "unit": "point*pixel/s", "cores": threads,
               "kind": "oracle",
               "sample": f"every {args.sample_row_step}th row ({len(rows)} rows x {W} columns) "
                         f"of the {W}x{H} hologram, all {N} points: {sample_pp:.3e} "
                         f"point*pixels in {dt:.1f} s (FP64, libm cos)"}
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
        import oracle as orc
        sph_ref = None
        for m, r in results.items():
            if m == "spherical_fp32":
                # Eq. (1) has its own reference: every 4th sample row
                srows = rows[::4]
                t0 = time.perf_counter()
                sph_ref = orc.spherical_complex(W, H, c.pitch, c.wavelength, c.x, c.y, c.z,
                                                c.amp, rows=srows, threads=threads)[0]
                dt = time.perf_counter() - t0
                spp = len(srows) * W * N
                r["cpu_baseline"] = {"value": spp / dt, "unit": "point*pixel/s", "cores": threads,
                                     "kind": "oracle",
                                     "sample": f"Eq. (1) with its imaginary part, every "
                                               f"{4 * args.sample_row_step}th row ({len(srows)} "
                                               f"rows x {W} columns), all {N} points: "
                                               f"{spp:.3e} point*pixels in {dt:.1f} s"}
                got, want = r["sample"][::4], sph_ref
            else:
                got, want = r["sample"], ref
            r["nrms"] = orc.nrms(got, want)
            r["max_err"] = orc.max_err(got, want)
            log(f"mode {m}: nrms {r['nrms']:.3e} max {r['max_err']:.3e}")

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
        "roofline": h.get("roofline"),
        "cpu_baseline": cpu,
        "modes": {m: {k: v for k, v in r.items() if k != "sample"} for m, r in results.items()},
        "batch": batch,
        "kinoform": kino,
        "fresnel_diffraction": fres,
        "large": large,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
