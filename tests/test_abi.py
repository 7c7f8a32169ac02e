"""The C-ABI library loads, exports what include/cgh.h declares, and rejects
bad arguments before touching the GPU (so these run on a host without one)."""
import ctypes
import os
import re

import pytest

import paper_1309_2734_amd as cgh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgh.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"CGH_API\s+[^;(]*?\b(cgh_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(cgh.LIB_PATH):
        from paper_1309_2734_amd import build
        build.build()
    return cgh.lib()


def test_header_declares_the_binding_exports():
    assert _declared_functions() == sorted(cgh.EXPORTS)


def test_every_declared_symbol_is_exported(L):
    for name in _declared_functions():
        assert hasattr(L, name), name
    # nothing else leaks out of the library
    out = os.popen(f"nm -D --defined-only {cgh.LIB_PATH}").read()
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == _declared_functions()


def test_strerror_and_version(L):
    assert L.cgh_strerror(0) == b"success"
    assert L.cgh_strerror(1) == b"invalid argument"
    assert L.cgh_strerror(5) == b"invalid call order"
    assert L.cgh_strerror(99) == b"unknown status"
    assert L.cgh_version() == 10100


def _create(L, w=64, h=32, p=8e-6, lam=5e-7, dev=0, null_out=False):
    out = ctypes.c_void_p(123)
    st = L.cgh_create(None if null_out else ctypes.byref(out), w, h, p, lam, dev)
    return st, out


@pytest.mark.parametrize("kw", [
    dict(null_out=True), dict(w=0), dict(h=0), dict(w=65537), dict(h=-3),
    dict(p=0.0), dict(p=-1e-6), dict(p=float("nan")), dict(p=float("inf")),
    dict(lam=0.0), dict(lam=float("nan")), dict(dev=-1),
])
def test_create_rejects_bad_arguments(L, kw):
    st, out = _create(L, **kw)
    assert st == cgh.EINVAL
    if not kw.get("null_out"):
        assert out.value is None       # *out is cleared on failure
    assert len(L.cgh_last_error()) > 0


def test_create_without_gpu_reports_device_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    st, out = _create(L)
    assert st == cgh.EDEVICE and out.value is None
    with pytest.raises(cgh.CghError) as e:
        cgh.Context(64, 32, 8e-6, 5e-7)
    assert e.value.status == cgh.EDEVICE


def test_null_context_is_rejected_everywhere(L):
    f = (cgh.Frame * 1)()
    assert L.cgh_points_upload(None, None, None, None, None, 0, 0, None) == cgh.EINVAL
    assert L.cgh_compute(None, 0, ctypes.c_void_p(16), None) == cgh.EINVAL
    assert L.cgh_compute_complex(None, 0, ctypes.c_void_p(16), None) == cgh.EINVAL
    assert L.cgh_kinoform(None, 0, ctypes.c_void_p(16), None) == cgh.EINVAL
    assert L.cgh_tune(None, 0, 1, None, 0, None) == cgh.EINVAL
    assert L.cgh_tune_batch(None, f, 1, 0, ctypes.c_void_p(16), 1, None, 0, None) == cgh.EINVAL
    assert L.cgh_fresnel_run(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == cgh.EINVAL
    L.cgh_fresnel_destroy(None)
    assert L.cgh_batch_compute(None, f, 1, 0, ctypes.c_void_p(16), None) == cgh.EINVAL
    assert L.cgh_wrm_record(None, 0.3, 64, ctypes.c_void_p(16), None) == cgh.EINVAL
    assert L.cgh_wrm_compute(None, None, ctypes.c_void_p(16), ctypes.c_void_p(16),
                             None) == cgh.EINVAL
    assert L.cgh_profile_enable(None, 1) == cgh.EINVAL
    assert L.cgh_profile_reset(None) == cgh.EINVAL
    cnt = ctypes.c_int32()
    assert L.cgh_profile_read(None, None, None, None, 0, ctypes.byref(cnt)) == cgh.EINVAL
    L.cgh_destroy(None)   # NULL-safe


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(cgh, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(cgh, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        cgh.lib()


@pytest.mark.parametrize("n, p, lam, z, dev", [
    (0, 8e-6, 5e-7, 0.1, 0), (48, 8e-6, 5e-7, 0.1, 0), (8, 8e-6, 5e-7, 0.1, 0),
    (16384, 8e-6, 5e-7, 0.1, 0), (64, 0.0, 5e-7, 0.1, 0), (64, 8e-6, float("nan"), 0.1, 0),
    (64, 8e-6, 5e-7, 0.0, 0), (64, 8e-6, 5e-7, float("inf"), 0), (64, 8e-6, 5e-7, 0.1, -1),
])
def test_fresnel_create_rejects_bad_arguments(L, n, p, lam, z, dev):
    out = ctypes.c_void_p(123)
    assert L.cgh_fresnel_create(ctypes.byref(out), n, p, lam, z, dev) == cgh.EINVAL
    assert out.value is None
    assert L.cgh_fresnel_create(None, 64, 8e-6, 5e-7, 0.1, 0) == cgh.EINVAL


def test_fresnel_create_without_gpu_reports_device_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    out = ctypes.c_void_p(123)
    assert L.cgh_fresnel_create(ctypes.byref(out), 64, 8e-6, 5e-7, 0.1, 0) == cgh.EDEVICE
    assert out.value is None


def test_binding_rejects_tensors_on_another_device():
    """Device tensors must sit on the context's (or plan's) device: the
    library writes through their pointers on its own device."""
    class _Dev:
        def __init__(self, i):
            self.index = i

    class _T:
        def __init__(self, i):
            self.device = _Dev(i)

    cgh._on_device(_T(0), 0, "out")
    with pytest.raises(ValueError, match="out is on"):
        cgh._on_device(_T(1), 0, "out")


def _noalloc(L, w=64, h=32, p=8e-6, lam=5e-7, pts=16, n=4, mode=0, out=16, dev=0):
    ptr = ctypes.c_void_p(pts) if pts else None
    return L.cgh_compute_noalloc(w, h, p, lam, ptr, ptr, ptr, ptr, n, mode,
                                 ctypes.c_void_p(out) if out else None, dev, None)


@pytest.mark.parametrize("kw", [
    dict(w=0), dict(h=65537), dict(p=0.0), dict(lam=float("inf")), dict(n=-1),
    dict(n=(1 << 34) + 1), dict(pts=0), dict(out=0), dict(mode=6), dict(mode=-1), dict(dev=-1),
    dict(dev=64),
    # the intermediates of one 32-point group exceed the 32 MiB array
    dict(w=65536, h=65536, mode=cgh.SEPARABLE_FP32), dict(w=65536, h=65536, mode=cgh.SPLIT_BF16),
    dict(w=65536, h=65536, mode=cgh.SPLIT_FP16), dict(w=65536, h=65536, mode=cgh.SPHERICAL_FP32),
])
def test_noalloc_rejects_bad_arguments_before_any_hip_call(L, kw):
    """Checked before the device is touched, so identical on a GPU-less host."""
    assert _noalloc(L, **kw) == cgh.EINVAL
    assert len(L.cgh_last_error()) > 0


def test_noalloc_largest_accepted_sizes_pass_the_checks(L):
    """The direct FP32 and one-product FP16 modes fit one 32-point group of a
    65536 x 65536 hologram into the static array, every mode fits 65536 x
    32768; without a
    GPU such calls then fail at the device, not at the argument checks."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    for mode in (cgh.DIRECT_FP32, cgh.FP16):
        assert _noalloc(L, w=65536, h=65536, mode=mode) == cgh.EDEVICE, mode
    for mode in range(6):
        assert _noalloc(L, w=65536, h=32768, mode=mode) == cgh.EDEVICE, mode
    assert _noalloc(L, n=0, pts=0) == cgh.EDEVICE
