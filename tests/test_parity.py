"""GPU parity: every evaluation mode of libcgh.so against the FP64 oracle.

Tolerances (normalised RMS error vs the FP64 oracle, over the evaluation set):
  direct FP32 .............. 1e-5
  separable FP32 (MFMA) .... 1e-5
  BF16 / FP16 hi+lo split .. 1e-3
  FP16 single product ...... 1e-3
The FP32 forms and the split forms are held to their target accuracies; the
single-product FP16 form is held to the split forms' bound.
Full-size workloads are compared on strided pixel subsets the oracle
evaluates pixel by pixel; small ones on the full grid.
"""
import os

import numpy as np
import pytest

import cghgen
import oracle
import paper_1309_2734_amd as cgh

pytestmark = pytest.mark.gpu

TOL = {cgh.DIRECT_FP32: 1e-5, cgh.SEPARABLE_FP32: 1e-5, cgh.SPLIT_BF16: 1e-3,
       cgh.SPLIT_FP16: 1e-3, cgh.FP16: 1e-3}
NAMES = {v: k for k, v in cgh.MODES.items()}
GEMM_MODES = (cgh.SPLIT_BF16, cgh.SPLIT_FP16, cgh.FP16, cgh.SEPARABLE_FP32)
ALL_MODES = (cgh.DIRECT_FP32,) + GEMM_MODES


_REFS = {}     # oracle references shared by parametrised cases


def say(*a):
    print("[parity]", *a, flush=True)


def gpu_hologram(cloud, mode, ctx=None):
    import torch
    own = ctx is None
    if own:
        ctx = cgh.Context(cloud.width, cloud.height, cloud.pitch, cloud.wavelength)
        ctx.upload_cloud(cloud)
    out = torch.empty((cloud.height, cloud.width), dtype=torch.float32, device="cuda")
    ctx.compute(out, mode)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.float64)
    if own:
        ctx.close()
    return res


def check(name, got, ref, mode):
    e = oracle.nrms(got, ref)
    m = oracle.max_err(got, ref)
    say(f"{name} {NAMES[mode]}: nrms={e:.3e} max={m:.3e}")
    assert np.all(np.isfinite(got))
    assert e <= TOL[mode], f"{name} {NAMES[mode]} nrms {e:.3e} > {TOL[mode]:.0e}"
    return e


# ------------------------------------------------------------ full grids
@pytest.mark.parametrize("mode", ALL_MODES, ids=[NAMES[m] for m in ALL_MODES])
def test_c1_full_grid(mode):
    c = cghgen.make_config(1)
    say(f"C1 {c.width}x{c.height} N={c.n} {NAMES[mode]}")
    ref = oracle.cloud_fresnel(c)
    got = gpu_hologram(c, mode)
    e = check("C1", got, ref, mode)
    if mode == cgh.DIRECT_FP32:
        assert e < 2e-6
    if mode in (cgh.SPLIT_BF16, cgh.SPLIT_FP16):
        assert e < 1e-4


def test_zone_plate_layout_and_orientation():
    """One point on a pixel centre with beta = 1/8 rev/px^2 (as in the oracle's
    closed-form pin): every mode must give cos(pi ((ix-ix0)^2+(iy-iy0)^2)/4),
    which fixes the row-major layout, orientation and centre convention.
    p = 2^-17 m, z = 2^-11 m and the point offsets are exact in float32, so
    the float32 inputs carry no rounding."""
    p, z = 2.0 ** -17, 2.0 ** -11
    lam = 4.0 * p * p / z          # 2^-21 m = 476.8 nm
    W, H = 97, 45
    ix0, iy0 = 48 + 7, 22 - 4
    c = cghgen.Cloud("zone", W, H, p, lam, np.array([7 * p], np.float32),
                     np.array([-4 * p], np.float32), np.array([z], np.float32),
                     np.array([1.0], np.float32))
    n = np.arange(W)[None, :] - ix0
    m = np.arange(H)[:, None] - iy0
    exp = np.cos(np.pi * ((n * n + m * m) % 8) / 4.0)
    for mode in ALL_MODES:
        say(f"zone plate {NAMES[mode]}")
        got = gpu_hologram(c, mode)
        tol = 2e-6 if mode == cgh.DIRECT_FP32 else (1e-2 if mode == cgh.FP16 else 1e-4)
        assert np.max(np.abs(got - exp)) < tol, NAMES[mode]


# ------------------------------------------------------- full-size samples
def _strided(c, step):
    cols = sorted(set(range(0, c.width, step)) | {c.width - 1})
    rows = sorted(set(range(0, c.height, step)) | {c.height - 1})
    return np.array(cols), np.array(rows)


# Full-size samples.  The matrix kernels' output fragments are 16 x 16 and the
# direct kernel's lanes own bands of 4-16 rows, so a sample whose stride is
# coprime to 16 (7, 9) reaches every fragment position and every row of a
# band; the evaluation sets of the workloads (every 8th row and column, or a
# crop) are checked as well.
@pytest.mark.parametrize("mode", ALL_MODES, ids=[NAMES[m] for m in ALL_MODES])
def test_c2_full_size_strided(mode):
    c = cghgen.make_config(2)
    cols, rows = _strided(c, 7)
    say(f"C2 {c.width}x{c.height} N={c.n} {NAMES[mode]} sample {len(rows)}x{len(cols)}")
    if "c2_7" not in _REFS:
        _REFS["c2_7"] = oracle.cloud_fresnel(c, cols=cols, rows=rows)
    got = gpu_hologram(c, mode)[np.ix_(rows, cols)]
    check("C2", got, _REFS["c2_7"], mode)


@pytest.mark.parametrize("mode", ALL_MODES, ids=[NAMES[m] for m in ALL_MODES])
def test_c2_full_size_tuned_shapes(mode):
    """The launch shape the tuner picks at 1920 x 1080 x 10,000 points (the
    benchmark's configuration), checked on every 9th row and column."""
    c = cghgen.make_config(2)
    cols, rows = _strided(c, 9)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    say(f"C2 tuned {NAMES[mode]}: {ctx.tune(mode, repeats=2)}")
    if "c2_9" not in _REFS:
        _REFS["c2_9"] = oracle.cloud_fresnel(c, cols=cols, rows=rows)
    got = gpu_hologram(c, mode, ctx)[np.ix_(rows, cols)]
    ctx.close()
    check("C2 tuned", got, _REFS["c2_9"], mode)


@pytest.mark.parametrize("mode", (cgh.DIRECT_FP32, cgh.SPLIT_BF16, cgh.SEPARABLE_FP32),
                         ids=["direct_fp32", "split_bf16", "separable_fp32"])
def test_c3_full_size_every_8th(mode):
    """2048 x 2048, 65,536 points, on its evaluation set: every 8th row and
    column (256 x 256 pixels, corners included)."""
    c = cghgen.make_config(3)
    cols, rows = cghgen.strided_pixels(c.width, c.height, 8)
    say(f"C3 {c.width}x{c.height} N={c.n} {NAMES[mode]} sample {len(rows)}x{len(cols)}")
    if "c3" not in _REFS:
        _REFS["c3"] = oracle.cloud_fresnel(c, cols=cols, rows=rows)
    got = gpu_hologram(c, mode)[np.ix_(rows, cols)]
    check("C3", got, _REFS["c3"], mode)


@pytest.mark.parametrize("mode", (cgh.SPLIT_BF16, cgh.SEPARABLE_FP32, cgh.DIRECT_FP32),
                         ids=["split_bf16", "separable_fp32", "direct_fp32"])
def test_c5_large_scene_chunked(mode):
    """4096 x 4096 at 4 um, 10^6 points on an ellipsoid surface: the factors
    or tables of the whole cloud exceed the workspace budget, so the cloud
    is evaluated in point chunks that accumulate into the output.  Checked
    on the central 64 x 64 pixels of the workload's centred 256 x 256 crop
    (rows and columns 2016 .. 2079) and on a sparse stride-161 grid."""
    c = cghgen.make_config(5)
    cols, rows = cghgen.crop_pixels(2016, 2016, 64, 64)
    scols, srows = np.arange(7, c.width, 161), np.arange(3, c.height, 161)
    say(f"C5 {c.width}x{c.height} N={c.n} {NAMES[mode]} crop {len(rows)}x{len(cols)}")
    if "c5" not in _REFS:
        _REFS["c5"] = oracle.cloud_fresnel(c, cols=cols, rows=rows)
        _REFS["c5s"] = oracle.cloud_fresnel(c, cols=scols, rows=srows)
    full = gpu_hologram(c, mode)
    check("C5 crop", full[np.ix_(rows, cols)], _REFS["c5"], mode)
    check("C5 sparse", full[np.ix_(srows, scols)], _REFS["c5s"], mode)


# ------------------------------------------------------------ edge cases
@pytest.mark.parametrize("n", [1, 2, 31, 33, 100])
def test_ragged_point_counts(n):
    c = cghgen.make_config(1, n=n)
    ref = oracle.cloud_fresnel(c)
    for mode in ALL_MODES:
        say(f"ragged N={n} {NAMES[mode]}")
        check(f"N={n}", gpu_hologram(c, mode), ref, mode)


@pytest.mark.parametrize("wh", [(1, 1), (65, 33), (300, 7), (7, 300), (129, 257)])
def test_ragged_hologram_sizes(wh):
    W, H = wh
    c0 = cghgen.make_config(1, n=77)
    c = cghgen.Cloud("ragged", W, H, c0.pitch, c0.wavelength, c0.x, c0.y, c0.z, c0.amp)
    ref = oracle.cloud_fresnel(c)
    for mode in ALL_MODES:
        say(f"size {W}x{H} {NAMES[mode]}")
        got = gpu_hologram(c, mode)
        if W * H == 1:
            assert abs(got[0, 0] - ref[0, 0]) <= TOL[mode] * max(1.0, abs(ref[0, 0])) * 10
        else:
            check(f"{W}x{H}", got, ref, mode)


@pytest.mark.parametrize("wh", [(65536, 5), (5, 65536)], ids=["65536x5", "5x65536"])
def test_maximum_width_and_height(wh):
    """The largest width (height) cgh_create accepts, with a thin other side:
    every index of a 65,536-pixel line, the last tiles of the padded table
    and factor layouts, and the widest launch grids.  Phases reach ~4e5
    revolutions at the far pixels, far past Nyquist, which the FP64 reduction
    must still hold."""
    W, H = wh
    c0 = cghgen.make_config(1, n=40)
    c = cghgen.Cloud("max", W, H, c0.pitch, c0.wavelength, c0.x, c0.y, c0.z, c0.amp)
    ref = oracle.cloud_fresnel(c)
    for mode in ALL_MODES:
        say(f"size {W}x{H} {NAMES[mode]}")
        check(f"{W}x{H}", gpu_hologram(c, mode), ref, mode)


def test_empty_cloud_and_zero_amplitudes_give_zero():
    import torch
    c = cghgen.make_config(1, n=40)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    for mode in ALL_MODES:
        say(f"empty cloud {NAMES[mode]}")
        ctx.upload(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32),
                   np.zeros(0, np.float32))
        out = torch.full((c.height, c.width), 7.0, device="cuda")
        ctx.compute(out, mode)
        assert torch.count_nonzero(out).item() == 0
        ctx.upload(c.x, c.y, c.z, np.zeros(c.n, np.float32))
        out.fill_(7.0)
        ctx.compute(out, mode)
        assert torch.count_nonzero(out).item() == 0
    ctx.close()


def test_point_chunking_matches_oracle(monkeypatch):
    """A workspace budget far below the cloud's needs forces many point
    chunks that accumulate into the output in order."""
    c = cghgen.make_config(1, n=3000)
    ref = oracle.cloud_fresnel(c, rows=range(0, 256, 3))
    monkeypatch.setenv("CGH_WORKSPACE_BYTES", str(1 << 20))
    for mode in ALL_MODES:
        say(f"chunked N=3000 {NAMES[mode]}")
        got = gpu_hologram(c, mode)[0::3]
        check("chunked", got, ref, mode)


@pytest.mark.parametrize("splits", [0, 2, 9, 11, 24], ids=lambda s: f"splits{s or '_auto'}")
def test_split_k_counts(splits, monkeypatch):
    """K split counts 2, 9, 11, 24 and the library's own (24 in BF16, 48 in
    FP32) on a small hologram of many points (one output tile), including a
    width that leaves the 4-wide reduce path."""
    for w, h in ((96, 80), (97, 80)):
        c0 = cghgen.make_config(1, n=3072)
        c = cghgen.Cloud("splits", w, h, c0.pitch, c0.wavelength, c0.x, c0.y, c0.z, c0.amp)
        key = f"splits{w}x{h}"
        if key not in _REFS:
            _REFS[key] = oracle.cloud_fresnel(c)
        if splits:
            monkeypatch.setenv("CGH_GEMM_PLAN", f"192,192,2,4,3,{splits}")
        for mode in (cgh.SPLIT_BF16, cgh.SEPARABLE_FP32):
            say(f"{w}x{h} N=3072 {NAMES[mode]} splits {splits or 'auto'}")
            check(f"splits={splits}", gpu_hologram(c, mode), _REFS[key], mode)


@pytest.mark.parametrize("splits,rows", [(2, "4"), (4, "16"), (4, "8")])
def test_direct_point_splits(splits, rows, monkeypatch):
    """The direct modes split over the points (runs of whole group pairs into
    partial planes, summed in a fixed order): the full-size 1920 x 1080 case,
    small clouds with fewer group pairs than splits, a chunked cloud, the
    exact spherical wave, and bitwise repeatability."""
    monkeypatch.setenv("CGH_DIRECT_SPLITS", str(splits))
    monkeypatch.setenv("CGH_DIRECT_ROWS", rows)
    c = cghgen.make_config(2)
    cols, rows_s = _strided(c, 8)
    key = "c2_strided8"
    if key not in _REFS:
        _REFS[key] = oracle.cloud_fresnel(c, cols=cols, rows=rows_s)
    say(f"direct splits {splits} rows {rows} C2")
    a = gpu_hologram(c, cgh.DIRECT_FP32)
    check(f"split {splits}", a[np.ix_(rows_s, cols)], _REFS[key], cgh.DIRECT_FP32)
    assert np.array_equal(a, gpu_hologram(c, cgh.DIRECT_FP32))
    for n in (1, 33, 100, 3000):
        s = cghgen.make_config(1, n=n)
        say(f"direct splits {splits} rows {rows} N={n}")
        check(f"split {splits} N={n}", gpu_hologram(s, cgh.DIRECT_FP32), oracle.cloud_fresnel(s),
              cgh.DIRECT_FP32)
    s = cghgen.make_config(1, n=500)
    sph = oracle.spherical_complex(s.width, s.height, s.pitch, s.wavelength, s.x, s.y, s.z,
                                   s.amp)[0]
    e = oracle.nrms(gpu_hologram(s, cgh.SPHERICAL_FP32), sph)
    say(f"spherical split {splits}: nrms={e:.3e}")
    assert e <= 1e-5
    monkeypatch.setenv("CGH_WORKSPACE_BYTES", str(1 << 20))
    s = cghgen.make_config(1, n=3000)
    check(f"split {splits} chunked", gpu_hologram(s, cgh.DIRECT_FP32), oracle.cloud_fresnel(s),
          cgh.DIRECT_FP32)


def test_bitwise_repeatable():
    c = cghgen.make_config(2, n=2000)
    for mode in ALL_MODES:
        say(f"repeat {NAMES[mode]}")
        a = gpu_hologram(c, mode)
        b = gpu_hologram(c, mode)
        assert np.array_equal(a, b), NAMES[mode]


def test_mirror_symmetry_on_gpu():
    c = cghgen.make_config(1, n=64)
    m = cghgen.Cloud("mirror", c.width, c.height, c.pitch, c.wavelength, -c.x, c.y, c.z, c.amp)
    for mode in ALL_MODES:
        say(f"mirror {NAMES[mode]}")
        a = gpu_hologram(c, mode)
        b = gpu_hologram(m, mode)
        assert oracle.nrms(b[:, ::-1], a) <= TOL[mode]


def test_device_upload_matches_host_upload():
    import torch
    c = cghgen.make_config(1, n=500)
    for mode in ALL_MODES:
        say(f"device upload {NAMES[mode]}")
        host = gpu_hologram(c, mode)
        ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
        ctx.upload(*[torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z, c.amp)])
        dev = gpu_hologram(c, mode, ctx)
        ctx.close()
        assert np.array_equal(host, dev)


# ------------------------------------------------------------ batches
def _batch_case():
    counts = [0, 1, 37, 500, 2000, 33, 700]
    return cghgen.make_batch(n_frames=len(counts), width=200, height=120, counts=counts)


@pytest.mark.parametrize("mode", ALL_MODES, ids=[NAMES[m] for m in ALL_MODES])
def test_batch_frames_match_oracle_and_single(mode, monkeypatch):
    import torch
    # the single evaluations below unsplit, as a batch frame is: a small
    # hologram's points are otherwise split into runs summed separately
    monkeypatch.setenv("CGH_DIRECT_SPLITS", "1")
    b = _batch_case()
    frames = cgh.batch_frames(b)
    # an overlapping frame and a repeated frame
    frames.append((int(b.offsets[3]) + 100, 1500, 532e-9))
    frames.append(frames[4])
    say(f"batch {len(frames)} frames {NAMES[mode]}")
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    out = torch.empty((len(frames), b.height, b.width), device="cuda")
    ctx.batch_compute(frames, out, mode)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    for f, (o, n, lam) in enumerate(frames):
        sl = slice(o, o + n)
        ref = oracle.fresnel(b.width, b.height, b.pitch, lam, b.x[sl], b.y[sl], b.z[sl],
                             b.amp[sl])
        if n == 0:
            assert np.all(got[f] == 0.0)
            continue
        check(f"batch frame {f} N={n}", got[f], ref, mode)
        # a single-hologram evaluation of that frame: the same numbers for the
        # (unsplit) direct kernel; the matrix-core batch runs each frame's whole K range
        # in one workgroup (no split-K), so its sums are ordered differently
        single = cgh.Context(b.width, b.height, b.pitch, lam)
        single.upload(b.x[sl], b.y[sl], b.z[sl], b.amp[sl])
        one = torch.empty((b.height, b.width), device="cuda")
        single.compute(one, mode)
        torch.cuda.synchronize()
        if mode == cgh.DIRECT_FP32:
            assert np.array_equal(one.cpu().numpy(), out[f].cpu().numpy()), f"frame {f}"
        else:
            assert oracle.nrms(out[f].cpu().numpy(), one.cpu().numpy()) < 1e-5, f"frame {f}"
        single.close()
    ctx.close()


@pytest.mark.parametrize("mode", ALL_MODES, ids=[NAMES[m] for m in ALL_MODES])
def test_batch_frame_groups_under_a_small_workspace(mode, monkeypatch):
    """A workspace budget below the batch's factors splits the frames into
    several groups (a frame larger than the budget alone in one), each with
    its own factor and GEMM launches.  Every frame matches the oracle; in the
    matrix-core modes a frame's sums do not depend on its group (one
    workgroup per output tile over the frame's whole K range), so the
    result equals the one-group batch bit for bit."""
    import torch
    b = _batch_case()
    frames = cgh.batch_frames(b)
    frames.append((int(b.offsets[3]) + 100, 1500, 633e-9))
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    F = len(frames)
    whole = torch.empty((F, b.height, b.width), device="cuda")
    ctx.batch_compute(frames, whole, mode)
    torch.cuda.synchronize()
    monkeypatch.setenv("CGH_WORKSPACE_BYTES", str(1 << 20))
    say(f"batch {F} frames in groups {NAMES[mode]}")
    out = torch.empty_like(whole)
    ctx.batch_compute(frames, out, mode)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    for f, (o, n, lam) in enumerate(frames):
        sl = slice(o, o + n)
        if n == 0:
            assert np.all(got[f] == 0.0)
            continue
        ref = oracle.fresnel(b.width, b.height, b.pitch, lam, b.x[sl], b.y[sl], b.z[sl],
                             b.amp[sl])
        check(f"grouped batch frame {f} N={n}", got[f], ref, mode)
    if mode != cgh.DIRECT_FP32:
        assert np.array_equal(out.cpu().numpy(), whole.cpu().numpy())
    ctx.close()


@pytest.mark.parametrize("mode", ALL_MODES, ids=[NAMES[m] for m in ALL_MODES])
def test_batch_graph_replays_match_eager(mode):
    """On a non-default stream a repeated batch call replays a captured HIP
    graph.  Replays, with eager work and synchronisations in between, must
    give the eager result bit for bit."""
    import torch
    b = _batch_case()
    frames = cgh.batch_frames(b)
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    F = len(frames)
    eager = torch.empty((F, b.height, b.width), device="cuda")
    ctx.batch_compute(frames, eager, mode)          # null stream: never captured
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    side = torch.cuda.Stream()
    out = torch.empty_like(eager)
    other = cghgen.make_config(1, n=50)
    octx = cgh.Context(other.width, other.height, other.pitch, other.wavelength)
    octx.upload_cloud(other)
    scratch = torch.empty((other.height, other.width), device="cuda")
    for rep in range(4):
        say(f"graph replay {rep} {NAMES[mode]}")
        out.fill_(-1.0)
        torch.cuda.synchronize()
        ctx.batch_compute(frames, out, mode, stream=side)
        side.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), f"replay {rep}"
        octx.compute(scratch, mode)                  # eager work between replays
        torch.cuda.synchronize()
    ctx.close()
    octx.close()


@pytest.mark.parametrize("mode", (cgh.SPLIT_FP16, cgh.FP16, cgh.DIRECT_FP32),
                         ids=["split_fp16", "fp16", "direct_fp32"])
def test_tune_batch_then_batch_matches_oracle(mode, tmp_path, monkeypatch):
    """cgh_tune_batch times every candidate launch of the batch, keeps the
    fastest under the batch's key (also in the cache file, which a new
    context reads back), and later batch calls -- eager and graph replays --
    use it and still match the oracle frame by frame."""
    import torch
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("CGH_TUNE_CACHE", str(cache))
    b = _batch_case()
    frames = cgh.batch_frames(b)
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    out = torch.empty((len(frames), b.height, b.width), device="cuda")
    rep = ctx.tune_batch(frames, out, mode, repeats=1)
    say(f"tune batch {NAMES[mode]}: {rep}")
    assert "/batch/" in rep and "(0 candidates)" not in rep
    assert "/batch/" in cache.read_text()
    side = torch.cuda.Stream()
    for rep_i in range(3):                        # eager, captured, replayed
        out.fill_(-1.0)
        torch.cuda.synchronize()
        ctx.batch_compute(frames, out, mode, stream=side)
        side.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        for f, (o, n, lam) in enumerate(frames):
            if n == 0:
                assert np.all(got[f] == 0.0)
                continue
            sl = slice(o, o + n)
            ref = oracle.fresnel(b.width, b.height, b.pitch, lam, b.x[sl], b.y[sl], b.z[sl],
                                 b.amp[sl])
            check(f"tuned batch frame {f} (call {rep_i})", got[f], ref, mode)
    ctx2 = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx2.upload_cloud(b)
    out2 = torch.empty_like(out)
    ctx2.batch_compute(frames, out2, mode)
    torch.cuda.synchronize()
    assert torch.equal(out2, out)                 # the cached choice, the same numbers
    ctx.close()
    ctx2.close()


@pytest.mark.parametrize("mode", (cgh.SPLIT_FP16, cgh.SPLIT_BF16, cgh.DIRECT_FP32,
                                  cgh.SEPARABLE_FP32),
                         ids=["split_fp16", "split_bf16", "direct_fp32", "separable_fp32"])
def test_batch_full_size_frames(mode):
    """Frames of the batch workload (1920 x 1080, RGB wavelengths, log-uniform
    point counts), the first six, each checked on its evaluation set: every
    8th row and column."""
    import torch
    b = cghgen.make_batch(n_frames=6)
    frames = cgh.batch_frames(b)
    say(f"batch 6 x 1920x1080 N={list(b.counts)} {NAMES[mode]}")
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    out = torch.empty((len(frames), b.height, b.width), device="cuda")
    ctx.batch_compute(frames, out, mode)
    torch.cuda.synchronize()
    cols, rows = cghgen.strided_pixels(b.width, b.height, 8)   # the workload's evaluation set
    for f, (o, n, lam) in enumerate(frames):
        sl = slice(o, o + n)
        ref = oracle.fresnel(b.width, b.height, b.pitch, lam, b.x[sl], b.y[sl], b.z[sl],
                             b.amp[sl], cols=cols, rows=rows)
        got = out[f].cpu().numpy().astype(np.float64)[np.ix_(rows, cols)]
        check(f"C4 frame {f} N={n}", got, ref, mode)
    ctx.close()


@pytest.mark.parametrize("mode", (cgh.SPLIT_FP16, cgh.FP16), ids=["split_fp16", "fp16"])
def test_batch_forced_192x320_tiles(mode, monkeypatch):
    """The persistent batch launch with 192 x 320 tiles (6 x 6 per 1920 x 1080
    frame): the first three frames of the batch workload on rows and columns
    at stride 7 (coprime to the MFMA blocks and the tiles)."""
    import torch
    monkeypatch.setenv("CGH_GEMM_PLAN", "192,320,2,4,2,0")
    b = cghgen.make_batch(n_frames=3)
    frames = cgh.batch_frames(b)
    say(f"batch 3 x 1920x1080 N={list(b.counts)} {NAMES[mode]} 192x320 tiles")
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    out = torch.empty((len(frames), b.height, b.width), device="cuda")
    ctx.batch_compute(frames, out, mode)
    torch.cuda.synchronize()
    cols, rows = np.arange(3, b.width, 7), np.arange(1, b.height, 7)
    for f, (o, n, lam) in enumerate(frames):
        sl = slice(o, o + n)
        ref = oracle.fresnel(b.width, b.height, b.pitch, lam, b.x[sl], b.y[sl], b.z[sl],
                             b.amp[sl], cols=cols, rows=rows)
        got = out[f].cpu().numpy().astype(np.float64)[np.ix_(rows, cols)]
        check(f"192x320 batch frame {f} N={n}", got, ref, mode)
    ctx.close()


def test_tune_picks_a_plan_and_caches_it(tmp_path, monkeypatch):
    import torch
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("CGH_TUNE_CACHE", str(cache))
    c = cghgen.make_config(1, n=4000)
    ref = oracle.cloud_fresnel(c, rows=range(0, 256, 5))
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    for mode in ALL_MODES:
        rep = ctx.tune(mode, repeats=2)
        say(f"tune {NAMES[mode]}: {rep}")
        assert "candidates" in rep and "(0 candidates)" not in rep
        got = gpu_hologram(c, mode, ctx)[0::5]
        check("tuned", got, ref, mode)
    lines = cache.read_text().splitlines()
    assert len(lines) == len(ALL_MODES)
    # a new context reads the cache back and evaluates with it
    ctx2 = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx2.upload_cloud(c)
    for mode in ALL_MODES:
        check("cached plan", gpu_hologram(c, mode, ctx2)[0::5], ref, mode)
    ctx.close()
    ctx2.close()


def test_tune_full_hd_covers_every_tile_shape():
    """Tuning at 1920 x 1080 tries tile shapes whose padding differs (1152 or
    1280 rows, 1920 or 2048 columns): the factors must be padded for the
    largest, then every tuned mode still matches the oracle."""
    c = cghgen.make_config(2, n=3000)
    cols, rows = np.arange(0, c.width, 40), np.arange(0, c.height, 40)
    ref = oracle.cloud_fresnel(c, cols=cols, rows=rows)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    for mode in ALL_MODES:
        say(f"tune full HD {NAMES[mode]}")
        say(ctx.tune(mode, repeats=1))
        got = gpu_hologram(c, mode, ctx)[np.ix_(rows, cols)]
        check("tuned full HD", got, ref, mode)
    ctx.close()


@pytest.mark.parametrize("plan", ["192,320,2,4,2,7", "192,320,2,4,2,3"])
def test_forced_192x320_tiles_full_hd(plan, monkeypatch):
    """The 192 x 320 tile shape at 1920 x 1080 (6 x 6 tiles, 1152 padded
    rows; 7 splits of 89-90 K blocks fill 252 workgroups) in every matrix
    mode, on rows and columns at stride 9 (coprime to the 16 x 16 MFMA
    blocks and the tiles)."""
    c = cghgen.make_config(2, n=3000)
    cols, rows = np.arange(4, c.width, 9), np.arange(2, c.height, 9)
    key = "c2_3000_stride9"
    if key not in _REFS:
        _REFS[key] = oracle.cloud_fresnel(c, cols=cols, rows=rows)
    monkeypatch.setenv("CGH_GEMM_PLAN", plan)
    for mode in GEMM_MODES:
        say(f"plan {plan} {NAMES[mode]} full HD")
        got = gpu_hologram(c, mode)[np.ix_(rows, cols)]
        check(f"plan {plan}", got, _REFS[key], mode)


# ------------------------------------------------------------ error paths
def test_error_paths_with_device():
    import torch
    c = cghgen.make_config(1, n=8)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    out = torch.empty((c.height, c.width), device="cuda")
    with pytest.raises(cgh.CghError) as e:
        ctx.compute(out, cgh.DIRECT_FP32)
    assert e.value.status == cgh.ESTATE
    bad_z = c.z.copy(); bad_z[3] = 0.0
    with pytest.raises(cgh.CghError) as e:
        ctx.upload(c.x, c.y, bad_z, c.amp)
    assert e.value.status == cgh.EINVAL
    bad_x = c.x.copy(); bad_x[0] = np.nan
    with pytest.raises(cgh.CghError) as e:
        ctx.upload(bad_x, c.y, c.z, c.amp)
    assert e.value.status == cgh.EINVAL
    ctx.upload_cloud(c)
    with pytest.raises(cgh.CghError) as e:
        ctx.compute(out, 17)
    assert e.value.status == cgh.EINVAL
    L = cgh.lib()
    assert L.cgh_compute(ctx._h, 0, None, None) == cgh.EINVAL
    with pytest.raises(cgh.CghError) as e:
        ctx.batch_compute([(5, 4, 5e-7)], out.view(1, c.height, c.width))
    assert e.value.status == cgh.EINVAL
    with pytest.raises(cgh.CghError) as e:
        ctx.batch_compute([(0, 4, -5e-7)], out.view(1, c.height, c.width))
    assert e.value.status == cgh.EINVAL
    f = (cgh.Frame * 1)()
    assert L.cgh_batch_compute(ctx._h, f, 0, 0, ctypes_ptr(out), None) == cgh.EINVAL
    ctx.close()


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())
