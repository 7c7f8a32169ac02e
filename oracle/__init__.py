"""FP64 CPU oracle for the point-cloud hologram (ctypes wrapper over cgh_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does, and this package never
imports the GPU library.  See cgh_oracle.c for what is computed and which
equations of the paper it follows (Section 2.1, Eq. (1), (2), (5); Section
2.3, Eq. (10) for the Fresnel diffraction of a sampled field).

Inputs are the float32 values handed to the GPU library, widened exactly to
float64, so input rounding is not counted as error.

Pins: every function here is checked in tests/test_oracle.py against closed
forms, invariants, an independent recurrence and 40-digit brute force.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cgh_oracle.c")
_LIB = os.path.join(_HERE, "libcgh_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off",
                        "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        for name in ("cgh_oracle_fresnel", "cgh_oracle_spherical"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                           ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int64, ip, ctypes.c_int64, ip,
                           dp, dp, ctypes.c_int32]
        fn = lib.cgh_oracle_wrm_record
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                       ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int64, ip, dp, dp, ctypes.c_int32]
        fn = lib.cgh_oracle_diffraction
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp,
                       ctypes.c_int64, ip, dp, dp, ctypes.c_int32]
        _lib = lib
    return _lib


def host_threads() -> int:
    """Threads the oracle uses by default: every core this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _eval(fn_name: str, width: int, height: int, pitch: float, wavelength: float,
          x, y, z, a, cols: Optional[Sequence[int]], rows: Optional[Sequence[int]],
          want_imag: bool, threads: Optional[int]):
    lib = _load()
    x64 = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    y64 = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
    z64 = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    a64 = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    n = x64.shape[0]
    if not (y64.shape[0] == n and z64.shape[0] == n and a64.shape[0] == n):
        raise ValueError("x, y, z, amp must have one length")
    c32 = np.ascontiguousarray(np.arange(width, dtype=np.int32) if cols is None
                               else np.asarray(cols, dtype=np.int32))
    r32 = np.ascontiguousarray(np.arange(height, dtype=np.int32) if rows is None
                               else np.asarray(rows, dtype=np.int32))
    re = np.zeros((r32.shape[0], c32.shape[0]), dtype=np.float64)
    im = np.zeros_like(re) if want_imag else None
    rc = getattr(lib, fn_name)(int(width), int(height), float(pitch), float(wavelength), n,
                               _dp(x64), _dp(y64), _dp(z64), _dp(a64),
                               c32.shape[0], _ip(c32), r32.shape[0], _ip(r32),
                               _dp(re), _dp(im) if im is not None else None,
                               int(threads or host_threads()))
    if rc != 0:
        raise RuntimeError(f"{fn_name} failed with code {rc}")
    return (re, im) if want_imag else re


def fresnel(width: int, height: int, pitch: float, wavelength: float, x, y, z, a,
            cols=None, rows=None, threads: Optional[int] = None) -> np.ndarray:
    """Amplitude hologram I[rows][cols] = sum_j A_j cos(pi r^2 / (lambda z_j)) in FP64.

    Eq. (5) with phi_r = 0, the 2 A_r factor and the per-point 2 pi z_j / lambda
    term dropped, under the Fresnel approximation of Eq. (2).  ``cols``/``rows``
    select the evaluation set (default: the full grid).
    """
    return _eval("cgh_oracle_fresnel", width, height, pitch, wavelength, x, y, z, a,
                 cols, rows, False, threads)


def fresnel_complex(width: int, height: int, pitch: float, wavelength: float, x, y, z, a,
                    cols=None, rows=None, threads: Optional[int] = None):
    """(Re O, Im O) of Eq. (2) without the per-point z_j term, FP64."""
    return _eval("cgh_oracle_fresnel", width, height, pitch, wavelength, x, y, z, a,
                 cols, rows, True, threads)


def spherical_complex(width: int, height: int, pitch: float, wavelength: float, x, y, z, a,
                      cols=None, rows=None, threads: Optional[int] = None):
    """(Re O, Im O) of Eq. (1): the exact spherical wave, phase 2 pi d / lambda."""
    return _eval("cgh_oracle_spherical", width, height, pitch, wavelength, x, y, z, a,
                 cols, rows, True, threads)


def cloud_fresnel(cloud, cols=None, rows=None, threads: Optional[int] = None) -> np.ndarray:
    """fresnel() for a cghgen.Cloud."""
    return fresnel(cloud.width, cloud.height, cloud.pitch, cloud.wavelength,
                   cloud.x, cloud.y, cloud.z, cloud.amp, cols, rows, threads)


def diffraction(u: np.ndarray, pitch: float, wavelength: float, z: float, rows=None,
                threads: Optional[int] = None) -> np.ndarray:
    """Eq. (10) by direct summation (cgh_oracle.c): the n x n complex field u
    propagated by z, read on the same grid; complex128 [len(rows), n]."""
    lib = _load()
    u = np.asarray(u)
    n = u.shape[0]
    if u.shape != (n, n):
        raise ValueError("u must be n x n")
    ur = np.ascontiguousarray(u.real, dtype=np.float64)
    ui = np.ascontiguousarray(u.imag, dtype=np.float64)
    r32 = np.ascontiguousarray(np.arange(n, dtype=np.int32) if rows is None
                               else np.asarray(rows, dtype=np.int32))
    re = np.zeros((r32.shape[0], n), dtype=np.float64)
    im = np.zeros_like(re)
    rc = lib.cgh_oracle_diffraction(int(n), float(pitch), float(wavelength), float(z), _dp(ur),
                                    _dp(ui), r32.shape[0], _ip(r32), _dp(re), _dp(im),
                                    int(threads or host_threads()))
    if rc != 0:
        raise RuntimeError(f"cgh_oracle_diffraction failed with code {rc}")
    return re + 1j * im


def wrm_record(n: int, pitch: float, wavelength: float, zw: float, x, y, z, a, rows=None,
               threads: Optional[int] = None) -> np.ndarray:
    """First step of the wavefront-recording method (cgh_oracle.c): the
    cloud's Fresnel wave recorded on the n x n virtual plane at distance zw
    from the hologram, each point (at d_j = z_j - zw > 0 beyond the plane)
    over its disc of radius lambda d_j / (2 p); complex128 [len(rows), n]."""
    lib = _load()
    arrs = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (x, y, z, a)]
    npts = arrs[0].shape[0]
    if any(v.shape[0] != npts for v in arrs):
        raise ValueError("x, y, z, amp must have one length")
    r32 = np.ascontiguousarray(np.arange(n, dtype=np.int32) if rows is None
                               else np.asarray(rows, dtype=np.int32))
    re = np.zeros((r32.shape[0], n), dtype=np.float64)
    im = np.zeros_like(re)
    rc = lib.cgh_oracle_wrm_record(int(n), float(pitch), float(wavelength), float(zw), npts,
                                   *[_dp(v) for v in arrs], r32.shape[0], _ip(r32), _dp(re),
                                   _dp(im), int(threads or host_threads()))
    if rc != 0:
        raise RuntimeError(f"cgh_oracle_wrm_record failed with code {rc}")
    return re + 1j * im


def diffraction_fft(u: np.ndarray, pitch: float, wavelength: float, z: float) -> np.ndarray:
    """Eq. (10) in its Fourier form: the field zero-padded to 2n x 2n, the
    impulse response h = exp(i pi (x^2 + y^2) / (lambda z)) sampled at the
    offsets -n .. n-1 in circular order, F^-1[F[u] F[h]] cropped to n x n, times
    exp(i 2 pi z / lambda) / (i lambda z) and the sample area p^2.  numpy FFTs
    in FP64 (Section 2.3)."""
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[0]
    m = 2 * n
    d = np.arange(m, dtype=np.float64)
    d = np.where(d < n, d, d - m)                       # circular offsets
    rev = np.fmod(d * d * (pitch * pitch / (2.0 * wavelength * z)), 1.0)
    h1 = np.exp(2j * np.pi * rev)                       # separable: h = h1 (x) h1
    up = np.zeros((m, m), dtype=np.complex128)
    up[:n, :n] = u
    spec = np.fft.fft2(up) * np.outer(np.fft.fft(h1), np.fft.fft(h1))
    o = np.fft.ifft2(spec)[:n, :n]
    zrev = np.fmod(z / wavelength, 1.0)
    pref = np.exp(2j * np.pi * zrev) / (1j * wavelength * z) * pitch * pitch
    return o * pref


def kinoform(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Phase-only hologram of Eq. (3): theta = atan2(Im O, Re O) wrapped to
    [0, 2 pi), quantised to 8 bits as floor(theta * 255 / (2 pi)).

    The quantisation is an integer decided by floating point, so it is taken
    in the precision the paper's program takes the argument in, FP32 (Section 4.1):
    the field is rounded to FP32, theta is the FP32 atan2 of it, 2 pi (FP32)
    is added when theta < 0, and the code is floor of theta times the FP32
    quotient 255 / (2 pi).  A device that decides in FP32 from the same FP32
    field agrees except within a few ulps of a code boundary, where either
    neighbour is correct.
    """
    r = np.asarray(re, dtype=np.float64).astype(np.float32)
    i = np.asarray(im, dtype=np.float64).astype(np.float32)
    theta = np.arctan2(i, r).astype(np.float32)
    two_pi = np.float32(6.28318530717958647692)
    theta = np.where(theta < np.float32(0.0), theta + two_pi, theta).astype(np.float32)
    codes_per_rad = np.float32(255.0) / two_pi
    code = np.floor((theta * codes_per_rad).astype(np.float32))
    return np.clip(code, 0, 255).astype(np.uint8)


def nrms(test: np.ndarray, ref: np.ndarray) -> float:
    """Normalised RMS error ||test - ref||_2 / ||ref||_2, in FP64."""
    t = np.asarray(test, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    den = float(np.sqrt(np.sum(r * r)))
    num = float(np.sqrt(np.sum((t - r) ** 2)))
    return num / den if den > 0 else num


def max_err(test: np.ndarray, ref: np.ndarray) -> float:
    """max |test - ref| / rms(ref), in FP64."""
    t = np.asarray(test, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    m = float(np.max(np.abs(t - r))) if r.size else 0.0
    return m / rms if rms > 0 else m
