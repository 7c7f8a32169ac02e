"""Python binding of libcgh.so, the gfx950 point-cloud hologram library.

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of the C library (include/cgh.h).  PyTorch supplies device memory and
streams; numpy arrays are accepted for host-side point uploads.

    import paper_1309_2734_amd as cgh
    ctx = cgh.Context(1920, 1080, pitch=8e-6, wavelength=532e-9)
    ctx.upload(x, y, z, amp)                     # float32 arrays (host or device)
    out = torch.empty((1080, 1920), device="cuda")
    ctx.compute(out, cgh.SPLIT_BF16)

The library must have been built (``python -m paper_1309_2734_amd.build``);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgh.so")

# cgh_mode
DIRECT_FP32 = 0
SPLIT_BF16 = 1
SPLIT_FP16 = 2
FP16 = 3
SEPARABLE_FP32 = 4
SPHERICAL_FP32 = 5      # the exact spherical wave (Eq. (1)), not the Fresnel sum
MODES = {"direct_fp32": DIRECT_FP32, "split_bf16": SPLIT_BF16, "split_fp16": SPLIT_FP16,
         "fp16": FP16, "separable_fp32": SEPARABLE_FP32, "spherical_fp32": SPHERICAL_FP32}

# cgh_status
OK, EINVAL, ENOMEM, EDEVICE, ENOTSUP, ESTATE = range(6)
STATUS_NAMES = {OK: "CGH_OK", EINVAL: "CGH_EINVAL", ENOMEM: "CGH_ENOMEM",
                EDEVICE: "CGH_EDEVICE", ENOTSUP: "CGH_ENOTSUP", ESTATE: "CGH_ESTATE"}

MEM_HOST = 0
MEM_DEVICE = 1

# every symbol include/cgh.h declares
EXPORTS = ("cgh_create", "cgh_points_upload", "cgh_compute", "cgh_compute_complex",
           "cgh_kinoform", "cgh_batch_compute", "cgh_compute_noalloc", "cgh_tune",
           "cgh_tune_batch",
           "cgh_fresnel_create", "cgh_wrm_record", "cgh_wrm_compute",
           "cgh_fresnel_run", "cgh_fresnel_destroy", "cgh_destroy", "cgh_strerror",
           "cgh_last_error", "cgh_profile_enable", "cgh_profile_reset", "cgh_profile_read",
           "cgh_version")


class CghError(RuntimeError):
    """A cgh_* call returned a status other than CGH_OK."""

    def __init__(self, status: int, call: str, detail: str):
        self.status = status
        super().__init__(f"{call}: {STATUS_NAMES.get(status, status)}: {detail}")


class Frame(ctypes.Structure):
    _fields_ = [("point_offset", ctypes.c_int64), ("point_count", ctypes.c_int64),
                ("wavelength", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcgh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1309_2734_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    st = ctypes.c_int
    L.cgh_create.argtypes = [ctypes.POINTER(vp), i32, i32, dbl, dbl, i32]
    L.cgh_create.restype = st
    L.cgh_points_upload.argtypes = [vp, vp, vp, vp, vp, i64, ctypes.c_int, vp]
    L.cgh_points_upload.restype = st
    L.cgh_compute.argtypes = [vp, ctypes.c_int, vp, vp]
    L.cgh_compute.restype = st
    L.cgh_compute_complex.argtypes = [vp, ctypes.c_int, vp, vp]
    L.cgh_compute_complex.restype = st
    L.cgh_kinoform.argtypes = [vp, ctypes.c_int, vp, vp]
    L.cgh_kinoform.restype = st
    L.cgh_batch_compute.argtypes = [vp, ctypes.POINTER(Frame), i32, ctypes.c_int, vp, vp]
    L.cgh_batch_compute.restype = st
    L.cgh_compute_noalloc.argtypes = [i32, i32, dbl, dbl, vp, vp, vp, vp, i64, ctypes.c_int, vp,
                                      i32, vp]
    L.cgh_compute_noalloc.restype = st
    L.cgh_tune.argtypes = [vp, ctypes.c_int, i32, ctypes.c_char_p, i32, vp]
    L.cgh_tune_batch.argtypes = [vp, ctypes.POINTER(Frame), i32, ctypes.c_int, vp, i32,
                                 ctypes.c_char_p, i32, vp]
    L.cgh_tune_batch.restype = st
    L.cgh_tune.restype = st
    L.cgh_destroy.argtypes = [vp]
    L.cgh_destroy.restype = None
    L.cgh_strerror.argtypes = [ctypes.c_int]
    L.cgh_strerror.restype = ctypes.c_char_p
    L.cgh_last_error.argtypes = []
    L.cgh_last_error.restype = ctypes.c_char_p
    L.cgh_profile_enable.argtypes = [vp, i32]
    L.cgh_profile_enable.restype = st
    L.cgh_profile_reset.argtypes = [vp]
    L.cgh_profile_reset.restype = st
    L.cgh_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i64),
                                   ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)]
    L.cgh_profile_read.restype = st
    L.cgh_version.argtypes = []
    L.cgh_version.restype = i32
    L.cgh_fresnel_create.argtypes = [ctypes.POINTER(vp), i32, dbl, dbl, dbl, i32]
    L.cgh_fresnel_create.restype = st
    L.cgh_fresnel_run.argtypes = [vp, vp, vp, vp]
    L.cgh_fresnel_run.restype = st
    L.cgh_fresnel_destroy.argtypes = [vp]
    L.cgh_fresnel_destroy.restype = None
    L.cgh_wrm_record.argtypes = [vp, dbl, i32, vp, vp]
    L.cgh_wrm_record.restype = st
    L.cgh_wrm_compute.argtypes = [vp, vp, vp, vp, vp]
    L.cgh_wrm_compute.restype = st
    _lib = L
    return L


def _check(status: int, call: str) -> None:
    if status != OK:
        detail = lib().cgh_last_error()
        raise CghError(status, call, detail.decode() if detail else "")


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _on_device(t, device: int, name: str) -> None:
    """Device tensors must live on the device of the context or plan."""
    if t.device.index != device:
        raise ValueError(f"{name} is on {t.device}, the library object on cuda:{device}")


def _stream_handle(stream, tensors: Iterable = ()) -> Optional[int]:
    """hipStream_t for a call: an explicit stream (torch.cuda.Stream or raw
    handle), else torch's current stream when device tensors take part."""
    if stream is not None:
        return int(getattr(stream, "cuda_stream", stream))
    for t in tensors:
        if _is_torch(t) and t.is_cuda:
            import torch
            return int(torch.cuda.current_stream(t.device).cuda_stream)
    return None


class Context:
    """One W x H hologram configuration on one device (a cgh_ctx)."""

    def __init__(self, width: int, height: int, pitch: float, wavelength: float,
                 device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().cgh_create(ctypes.byref(h), int(width), int(height), float(pitch),
                                float(wavelength), int(device)), "cgh_create")
        self._h = h
        self.width, self.height = int(width), int(height)
        self.pitch, self.wavelength, self.device = float(pitch), float(wavelength), int(device)
        self._keep = None

    # -- lifetime
    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().cgh_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- points
    def upload(self, x, y, z, amp, stream=None) -> None:
        """Copy a float32 SoA point cloud into the library (host numpy / CPU
        tensors: complete on return; CUDA tensors: ordered on the stream)."""
        arrs = [x, y, z, amp]
        if all(_is_torch(a) and a.is_cuda for a in arrs):
            import torch
            for a, name in zip(arrs, ("x", "y", "z", "amp")):
                _on_device(a, self.device, name)
            ts = [a.detach().to(torch.float32).contiguous() for a in arrs]
            n = ts[0].numel()
            if any(t.numel() != n for t in ts):
                raise ValueError("x, y, z, amp must have one length")
            self._keep = ts   # keep alive until the stream has copied them
            _check(lib().cgh_points_upload(self._h, *[t.data_ptr() for t in ts], n, MEM_DEVICE,
                                           _stream_handle(stream, ts)), "cgh_points_upload")
            return
        hs = [np.ascontiguousarray(a.detach().cpu().numpy() if _is_torch(a) else a,
                                   dtype=np.float32) for a in arrs]
        n = hs[0].shape[0]
        if any(h.ndim != 1 or h.shape[0] != n for h in hs):
            raise ValueError("x, y, z, amp must be 1-D arrays of one length")
        ptrs = [h.ctypes.data if n else None for h in hs]
        _check(lib().cgh_points_upload(self._h, *ptrs, n, MEM_HOST, _stream_handle(stream)),
               "cgh_points_upload")

    def upload_cloud(self, cloud, stream=None) -> None:
        """upload() the arrays of a cghgen.Cloud / Batch."""
        self.upload(cloud.x, cloud.y, cloud.z, cloud.amp, stream)

    # -- evaluation
    def _out_ptr(self, out, planes: int, dtype: str = "float32") -> int:
        if not (_is_torch(out) and out.is_cuda):
            raise TypeError(f"out must be a CUDA {dtype} torch tensor")
        import torch
        if out.dtype != getattr(torch, dtype) or not out.is_contiguous():
            raise TypeError(f"out must be contiguous {dtype}")
        if out.numel() != planes * self.width * self.height:
            raise ValueError(f"out must hold {planes} x {self.height} x {self.width} values")
        _on_device(out, self.device, "out")
        return out.data_ptr()

    def compute(self, out, mode: int = DIRECT_FP32, stream=None):
        """Hologram of the uploaded cloud into `out` ([H, W] float32, device)."""
        _check(lib().cgh_compute(self._h, int(mode), self._out_ptr(out, 1),
                                 _stream_handle(stream, [out])), "cgh_compute")
        return out

    def compute_complex(self, out, mode: int = DIRECT_FP32, stream=None):
        """Complex object wave into `out` ([2, H, W] float32, device): plane 0
        the real part (the hologram of compute()), plane 1 the imaginary part."""
        _check(lib().cgh_compute_complex(self._h, int(mode), self._out_ptr(out, 2),
                                         _stream_handle(stream, [out])), "cgh_compute_complex")
        return out

    def kinoform(self, out, mode: int = DIRECT_FP32, stream=None):
        """Phase-only hologram into `out` ([H, W] uint8, device)."""
        _check(lib().cgh_kinoform(self._h, int(mode), self._out_ptr(out, 1, "uint8"),
                                  _stream_handle(stream, [out])), "cgh_kinoform")
        return out

    def batch_compute(self, frames: Sequence[Tuple[int, int, float]], out,
                      mode: int = DIRECT_FP32, stream=None):
        """Holograms of frames (offset, count, wavelength) into out [F, H, W]."""
        F = len(frames)
        arr = (Frame * max(F, 1))()
        for i, (o, c, lam) in enumerate(frames):
            arr[i] = Frame(int(o), int(c), float(lam))
        _check(lib().cgh_batch_compute(self._h, arr, F, int(mode), self._out_ptr(out, F),
                                       _stream_handle(stream, [out])), "cgh_batch_compute")
        return out

    def tune(self, mode: int, repeats: int = 5, stream=None) -> str:
        """Autotune `mode`'s launch shape on the uploaded cloud (cgh_tune);
        returns the library's one-line report of the choice."""
        buf = ctypes.create_string_buffer(512)
        _check(lib().cgh_tune(self._h, int(mode), int(repeats), buf, 512,
                              _stream_handle(stream)), "cgh_tune")
        return buf.value.decode()

    def tune_batch(self, frames: Sequence[Tuple[int, int, float]], out, mode: int,
                   repeats: int = 3, stream=None) -> str:
        """Autotune the batched launch of `mode` for these frames
        (cgh_tune_batch; writes into `out` [F, H, W]); returns the report."""
        F = len(frames)
        arr = (Frame * max(F, 1))()
        for i, (o, c, lam) in enumerate(frames):
            arr[i] = Frame(int(o), int(c), float(lam))
        buf = ctypes.create_string_buffer(512)
        _check(lib().cgh_tune_batch(self._h, arr, F, int(mode), self._out_ptr(out, F),
                                    int(repeats), buf, 512, _stream_handle(stream, [out])),
               "cgh_tune_batch")
        return buf.value.decode()

    # -- wavefront recording (Section 2.3)
    def wrm_record(self, plane_z: float, field, stream=None):
        """Step 1: the cloud recorded on the n x n virtual plane at distance
        plane_z from the hologram, into `field` (CUDA complex64 [n, n])."""
        n = _plane_size(field)
        _on_device(field, self.device, "field")
        _check(lib().cgh_wrm_record(self._h, float(plane_z), n, field.data_ptr(),
                                    _stream_handle(stream, [field])), "cgh_wrm_record")
        return field

    def wrm_compute(self, plan: "FresnelPlan", field, out, stream=None):
        """Both steps: record on the plan's plane (distance plan.z) into
        `field`, propagate it with the plan, and write Re O over the
        hologram's window into `out` ([H, W] float32)."""
        if _plane_size(field) != plan.n:
            raise ValueError(f"field must be ({plan.n}, {plan.n})")
        _on_device(field, self.device, "field")
        _check(lib().cgh_wrm_compute(self._h, plan._h, field.data_ptr(), self._out_ptr(out, 1),
                                     _stream_handle(stream, [out])), "cgh_wrm_compute")
        return out

    # -- measurement
    def profile(self, on: bool = True) -> None:
        _check(lib().cgh_profile_enable(self._h, 1 if on else 0), "cgh_profile_enable")

    def profile_reset(self) -> None:
        _check(lib().cgh_profile_reset(self._h), "cgh_profile_reset")

    def profile_read(self) -> dict:
        """{kernel name: (launches, total ms)} since the last reset."""
        cap = 32
        names = (ctypes.c_char_p * cap)()
        launches = (ctypes.c_int64 * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = ctypes.c_int32()
        _check(lib().cgh_profile_read(self._h, names, launches, ms, cap, ctypes.byref(cnt)),
               "cgh_profile_read")
        return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(cnt.value)}


def _plane_size(field) -> int:
    import torch
    if not (_is_torch(field) and field.is_cuda and field.dtype == torch.complex64 and
            field.is_contiguous() and field.dim() == 2 and field.shape[0] == field.shape[1]):
        raise TypeError("field must be a contiguous square CUDA complex64 tensor")
    return int(field.shape[0])


class FresnelPlan:
    """Fresnel diffraction of n x n sampled fields by z (cgh_fresnel_*)."""

    def __init__(self, n: int, pitch: float, wavelength: float, z: float, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().cgh_fresnel_create(ctypes.byref(h), int(n), float(pitch), float(wavelength),
                                        float(z), int(device)), "cgh_fresnel_create")
        self._h = h
        self.n, self.pitch, self.wavelength, self.z = int(n), float(pitch), float(wavelength), float(z)
        self.device = int(device)

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().cgh_fresnel_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, u, out, stream=None):
        """Propagate u into out: CUDA complex64 tensors of shape [n, n]."""
        import torch
        for t, name in ((u, "u"), (out, "out")):
            if not (_is_torch(t) and t.is_cuda and t.dtype == torch.complex64 and t.is_contiguous()
                    and tuple(t.shape) == (self.n, self.n)):
                raise TypeError(f"{name} must be a contiguous CUDA complex64 tensor of shape "
                                f"({self.n}, {self.n})")
            _on_device(t, self.device, name)
        _check(lib().cgh_fresnel_run(self._h, u.data_ptr(), out.data_ptr(),
                                     _stream_handle(stream, [out])), "cgh_fresnel_run")
        return out


def compute_noalloc(out, x, y, z, amp, width: int, height: int, pitch: float, wavelength: float,
                    mode: int = DIRECT_FP32, device: int = 0, stream=None):
    """cgh_compute_noalloc: the hologram of the points x, y, z, amp (CUDA
    float32 tensors of one length) into `out` ([height, width] float32,
    CUDA), evaluated in the library's static scratch with no allocation."""
    import torch
    pts = [x, y, z, amp]
    for t, name in zip(pts, ("x", "y", "z", "amp")):
        if not (_is_torch(t) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                and t.dim() == 1):
            raise TypeError(f"{name} must be a contiguous 1-D CUDA float32 tensor")
        _on_device(t, device, name)
    n = x.numel()
    if any(t.numel() != n for t in pts):
        raise ValueError("x, y, z, amp must have one length")
    if not (_is_torch(out) and out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
            and out.numel() == int(width) * int(height)):
        raise TypeError("out must be a contiguous CUDA float32 tensor of height x width values")
    _on_device(out, device, "out")
    _check(lib().cgh_compute_noalloc(int(width), int(height), float(pitch), float(wavelength),
                                     *[t.data_ptr() if n else None for t in pts], n, int(mode),
                                     out.data_ptr(), int(device), _stream_handle(stream, [out])),
           "cgh_compute_noalloc")
    return out


def version() -> int:
    return int(lib().cgh_version())


def batch_frames(batch) -> list:
    """(offset, count, wavelength) triples of a cghgen.Batch."""
    return [(int(o), int(c), float(l)) for o, c, l in
            zip(batch.offsets, batch.counts, batch.wavelengths)]
