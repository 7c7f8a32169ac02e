"""GPU parity of the complex object wave (Eq. (2)) and of the phase-only
hologram of Eq. (3), every mode, against the FP64 oracle.

Complex field: both planes within the mode's NRMS bound, the real plane the
same as the amplitude hologram of cgh_compute.

Kinoform codes are an integer decided by floating point; both sides decide
in FP32, the paper's precision, so:
  - on the device's own field, the codes must equal the oracle's FP32
    quantisation of that field wherever the scaled phase theta * 255 / (2 pi)
    lies more than 1e-4 of a code (a few FP32 ulps) from a code boundary
    (device and host atan2 may differ by an ulp or two); nearer a boundary
    either neighbour is accepted (the wrap boundary joins codes 254/255
    and 0);
  - against the oracle's own FP64 field, the codes must agree wherever the
    device field's measured maximum error e cannot move the phase across a
    code boundary (the oracle's scaled phase is more than
    2 asin(e / |O|) * 255 / (2 pi) + 1e-3 from one), on at least half the
    pixels.
"""
import numpy as np
import pytest

import cghgen
import oracle
import paper_1309_2734_amd as cgh

pytestmark = pytest.mark.gpu

TOL = {cgh.DIRECT_FP32: 1e-5, cgh.SEPARABLE_FP32: 1e-5, cgh.SPLIT_BF16: 1e-3,
       cgh.SPLIT_FP16: 1e-3, cgh.FP16: 1e-3}
NAMES = {v: k for k, v in cgh.MODES.items()}
ALL_MODES = (cgh.DIRECT_FP32, cgh.SPLIT_BF16, cgh.SPLIT_FP16, cgh.FP16, cgh.SEPARABLE_FP32)
IDS = [NAMES[m] for m in ALL_MODES]
CODES_PER_RAD = 255.0 / (2.0 * np.pi)


def say(*a):
    print("[complex]", *a, flush=True)


def gpu_complex(ctx, c, mode):
    import torch
    out = torch.empty((2, c.height, c.width), dtype=torch.float32, device="cuda")
    ctx.compute_complex(out, mode)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_kinoform(ctx, c, mode):
    import torch
    out = torch.empty((c.height, c.width), dtype=torch.uint8, device="cuda")
    ctx.kinoform(out, mode)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def scaled_phase(re, im):
    th = np.arctan2(np.asarray(im, np.float64), np.asarray(re, np.float64))
    th = np.where(th < 0.0, th + 2.0 * np.pi, th)
    return th * CODES_PER_RAD


def check_codes_on_own_field(codes, re, im):
    t = scaled_phase(re, im)
    exact = oracle.kinoform(np.asarray(re, np.float64), np.asarray(im, np.float64))
    d = t - np.round(t)
    far = np.abs(d) > 1e-4
    assert np.array_equal(codes[far], exact[far]), \
        f"{int(np.sum(codes[far] != exact[far]))} codes differ away from boundaries"
    near = ~far
    k = np.round(t[near]).astype(np.int64)            # the boundary between k-1 and k
    ok = (codes[near] == (k % 255)) | (codes[near] == k - 1) | \
         ((k >= 255) & (codes[near] >= 254)) | ((k == 0) & (codes[near] >= 254))
    assert np.all(ok), "a code next to a boundary is neither neighbour"
    return int(np.sum(near))


def check_codes_against_oracle(codes, ref_re, ref_im, got_re, got_im):
    """Codes vs the oracle's FP64 field where the device field's measured
    error cannot move the phase across a code boundary: a field error of at
    most e moves the phase of O by at most asin(e / |O|)."""
    t = scaled_phase(ref_re, ref_im)
    mag = np.hypot(ref_re, ref_im)
    e = float(np.max(np.hypot(np.asarray(got_re, np.float64) - ref_re,
                              np.asarray(got_im, np.float64) - ref_im)))
    ratio = np.where(mag > 0, e / np.maximum(mag, 1e-300), np.inf)
    margin = np.where(ratio < 0.5, 2.0 * np.arcsin(np.minimum(ratio, 0.5)) * CODES_PER_RAD,
                      np.inf) + 1e-3
    d = t - np.round(t)
    sure = np.abs(d) > margin
    ref_codes = oracle.kinoform(ref_re, ref_im)
    bad = int(np.sum(codes[sure] != ref_codes[sure]))
    assert bad == 0, f"{bad} of {int(np.sum(sure))} well-conditioned codes differ"
    assert np.sum(sure) > 0.5 * codes.size, f"only {int(np.sum(sure))} codes checked"
    return int(np.sum(sure))


@pytest.mark.parametrize("mode", ALL_MODES, ids=IDS)
def test_c1_complex_field_and_kinoform(mode):
    import torch
    c = cghgen.make_config(1)
    say(f"C1 complex {NAMES[mode]}")
    re, im = oracle.fresnel_complex(c.width, c.height, c.pitch, c.wavelength,
                                    c.x, c.y, c.z, c.amp)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    got = gpu_complex(ctx, c, mode)
    for plane, ref, name in ((0, re, "Re"), (1, im, "Im")):
        e = oracle.nrms(got[plane], ref)
        say(f"  {name} nrms {e:.3e}")
        assert np.all(np.isfinite(got[plane]))
        assert e <= TOL[mode], f"{name} nrms {e:.3e}"
    # the real plane is the amplitude hologram
    amp = torch.empty((c.height, c.width), device="cuda")
    ctx.compute(amp, mode)
    torch.cuda.synchronize()
    amp = amp.cpu().numpy()
    if mode == cgh.DIRECT_FP32:
        assert np.array_equal(got[0], amp)
    else:
        assert oracle.nrms(got[0], amp) < 1e-5
    codes = gpu_kinoform(ctx, c, mode)
    near = check_codes_on_own_field(codes, got[0], got[1])
    sure = check_codes_against_oracle(codes, re, im, got[0], got[1])
    say(f"  kinoform: {near} pixels near a boundary, {sure} checked against the oracle")
    ctx.close()


@pytest.mark.parametrize("mode", ALL_MODES, ids=IDS)
def test_c2_complex_strided(mode):
    c = cghgen.make_config(2)
    cols, rows = np.arange(0, c.width, 48), np.arange(5, c.height, 48)
    say(f"C2 complex {NAMES[mode]}")
    re, im = oracle.fresnel_complex(c.width, c.height, c.pitch, c.wavelength,
                                    c.x, c.y, c.z, c.amp, cols=cols, rows=rows)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    got = gpu_complex(ctx, c, mode)[:, rows][:, :, cols]
    for plane, ref, name in ((0, re, "Re"), (1, im, "Im")):
        e = oracle.nrms(got[plane], ref)
        say(f"  {name} nrms {e:.3e}")
        assert e <= TOL[mode], f"{name} nrms {e:.3e}"
    codes = gpu_kinoform(ctx, c, mode)[np.ix_(rows, cols)]
    check_codes_on_own_field(codes, got[0], got[1])
    check_codes_against_oracle(codes, re, im, got[0], got[1])
    ctx.close()


@pytest.mark.parametrize("wh", [(1, 1), (65, 33), (7, 300), (129, 257)])
def test_ragged_sizes_complex(wh):
    """Odd sizes: the stacked factor's real/imaginary seam falls inside an
    operand block, and the kinoform's vector path has a ragged tail."""
    w, h = wh
    c0 = cghgen.make_config(1, n=77)
    c = cghgen.Cloud("ragged", w, h, c0.pitch, c0.wavelength, c0.x, c0.y, c0.z, c0.amp)
    re, im = oracle.fresnel_complex(w, h, c.pitch, c.wavelength, c.x, c.y, c.z, c.amp)
    ctx = cgh.Context(w, h, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    for mode in ALL_MODES:
        say(f"ragged {w}x{h} {NAMES[mode]}")
        got = gpu_complex(ctx, c, mode)
        if w * h > 1:
            assert oracle.nrms(got[0], re) <= TOL[mode]
            assert oracle.nrms(got[1], im) <= TOL[mode]
        else:
            assert abs(got[0, 0, 0] - re[0, 0]) <= 10 * TOL[mode] * max(1.0, abs(re[0, 0]))
            assert abs(got[1, 0, 0] - im[0, 0]) <= 10 * TOL[mode] * max(1.0, abs(im[0, 0]))
        check_codes_on_own_field(gpu_kinoform(ctx, c, mode), got[0], got[1])
    ctx.close()


def test_complex_chunked_matches_oracle(monkeypatch):
    """A workspace budget small enough to cut the cloud into point chunks:
    the chunks accumulate into both planes."""
    monkeypatch.setenv("CGH_WORKSPACE_BYTES", str(1 << 20))
    c = cghgen.make_config(1, n=3000)
    re, im = oracle.fresnel_complex(c.width, c.height, c.pitch, c.wavelength,
                                    c.x, c.y, c.z, c.amp)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    for mode in ALL_MODES:
        say(f"chunked complex {NAMES[mode]}")
        got = gpu_complex(ctx, c, mode)
        assert oracle.nrms(got[0], re) <= TOL[mode]
        assert oracle.nrms(got[1], im) <= TOL[mode]
    ctx.close()


def test_kinoform_output_checks():
    import torch
    c = cghgen.make_config(1, n=8)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    out = torch.empty((c.height, c.width), dtype=torch.uint8, device="cuda")
    with pytest.raises(cgh.CghError) as e:
        ctx.kinoform(out)
    assert e.value.status == cgh.ESTATE
    ctx.upload_cloud(c)
    with pytest.raises(TypeError):
        ctx.kinoform(torch.empty((c.height, c.width), device="cuda"))
    with pytest.raises(ValueError):
        ctx.compute_complex(torch.empty((c.height, c.width), device="cuda"))
    ctx.close()
