"""Seeded synthetic point clouds for the point-cloud hologram workloads.

This module only draws random inputs.  It holds none of the hologram
arithmetic: it is shared by the FP64 oracle (``oracle/``), the tests and the
benchmark, and the GPU library never imports it.

The paper's own test object (an 11,646-point model, Section 5) is not
available, so these clouds stand in for it.  The shapes follow the paper's
direct-calculation workload (1920x1080 hologram, 8 um pitch, 10^3..10^5
points; Section 4.1 and Table 5); the point distributions, depth ranges and
wavelengths are synthetic choices because the paper does not state them.

Conventions
-----------
* SI metres.  x, y are measured from the hologram centre; z > 0 is the
  distance from the hologram plane.
* Every draw is numpy PCG64 (``default_rng(seed)``), done in float64 in the
  order x, y, z, amplitude (one length-N vector each), then cast to float32:
  the float32 values are the inputs both the GPU path and the oracle see.
* Seed = configuration number (1..5); frame f of the batch workload uses
  seed 400 + f; the wavefront-recording workload uses seed 7.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = ["Cloud", "Batch", "make_config", "make_batch", "make_wrm", "uniform_cloud",
           "ellipsoid_cloud", "CONFIG_NAMES", "BATCH_WAVELENGTHS", "WRM_PLANE_Z", "WRM_PLANE_N"]


@dataclass
class Cloud:
    """One hologram's problem: grid, optics and a float32 SoA point cloud."""
    name: str
    width: int
    height: int
    pitch: float
    wavelength: float
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    amp: np.ndarray
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def point_pixels(self) -> int:
        return int(self.width) * int(self.height) * self.n


@dataclass
class Batch:
    """Many holograms of one size: frames pack their points back to back."""
    name: str
    width: int
    height: int
    pitch: float
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    amp: np.ndarray
    offsets: np.ndarray          # int64 [F]: first point of frame f
    counts: np.ndarray           # int64 [F]: points in frame f
    wavelengths: np.ndarray      # float64 [F]
    seeds: List[int] = field(default_factory=list)

    @property
    def n_frames(self) -> int:
        return int(self.offsets.shape[0])

    @property
    def point_pixels(self) -> int:
        return int(self.width) * int(self.height) * int(self.counts.sum())

    def frame(self, f: int) -> Cloud:
        o, c = int(self.offsets[f]), int(self.counts[f])
        return Cloud(f"{self.name}[{f}]", self.width, self.height, self.pitch,
                     float(self.wavelengths[f]), self.x[o:o + c], self.y[o:o + c],
                     self.z[o:o + c], self.amp[o:o + c],
                     self.seeds[f] if self.seeds else 0)


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64).astype(np.float32)


def uniform_cloud(name: str, width: int, height: int, pitch: float, wavelength: float,
                  n: int, xy_half: float, z_lo: float, z_hi: float,
                  amp_lo: float, amp_hi: float, seed: int) -> Cloud:
    """x, y ~ U(-xy_half, xy_half); z ~ U[z_lo, z_hi]; amplitude ~ U[amp_lo, amp_hi]."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-xy_half, xy_half, n)
    y = rng.uniform(-xy_half, xy_half, n)
    z = rng.uniform(z_lo, z_hi, n)
    a = rng.uniform(amp_lo, amp_hi, n)
    return Cloud(name, width, height, pitch, wavelength, _f32(x), _f32(y), _f32(z), _f32(a), seed)


def ellipsoid_cloud(name: str, width: int, height: int, pitch: float, wavelength: float,
                    n: int, semi_axes=(3e-3, 2e-3, 1e-3), centre=(0.0, 0.0, 0.5),
                    amp_lo: float = 0.5, amp_hi: float = 1.0, seed: int = 5) -> Cloud:
    """Points spread uniformly by area over a randomly rotated ellipsoid surface.

    Area-uniform sampling by rejection: u uniform on the unit sphere maps to
    D u (D = diag(semi_axes)); the surface element there scales with
    |D^-1 u| * abc, so accepting with probability |D^-1 u| * min(semi_axes)
    (always <= 1) makes the accepted points area-uniform.  The rotation is
    Haar-random (QR of a 3x3 Gaussian, signs fixed by diag(R)).  The
    amplitudes are drawn after the geometry.
    """
    rng = np.random.default_rng(seed)
    d = np.asarray(semi_axes, dtype=np.float64)
    g = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))
    pts = np.empty((0, 3))
    while pts.shape[0] < n:
        m = 2 * (n - pts.shape[0]) + 1024
        u = rng.standard_normal((m, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        w = np.linalg.norm(u / d, axis=1) * d.min()
        keep = rng.uniform(0.0, 1.0, m) < w
        pts = np.concatenate([pts, u[keep] * d])
    pts = pts[:n] @ q.T + np.asarray(centre, dtype=np.float64)
    a = rng.uniform(amp_lo, amp_hi, n)
    return Cloud(name, width, height, pitch, wavelength, _f32(pts[:, 0]), _f32(pts[:, 1]),
                 _f32(pts[:, 2]), _f32(a), seed,
                 {"rotation": q, "semi_axes": d, "centre": np.asarray(centre, dtype=np.float64)})


CONFIG_NAMES = {
    1: "C1 256x256 p=8um 632.8nm N=128",
    2: "C2 1920x1080 p=8um 532nm N=10000",
    3: "C3 2048x2048 p=8um 532nm N=65536",
    4: "C4 64x(1920x1080) p=8um RGB N_f log-uniform[1e3,5e4]",
    5: "C5 4096x4096 p=4um 532nm N=1e6 ellipsoid",
}

# Red, green and blue wavelengths cycled over the frames of a batch.
BATCH_WAVELENGTHS = (633e-9, 532e-9, 473e-9)


def make_config(k: int, n: Optional[int] = None, seed: Optional[int] = None) -> Cloud:
    """Single-hologram workloads 1, 2, 3 and 5 (4 is a batch: use make_batch).

    ``n`` overrides the point count (same distribution) for reduced-size
    tests; ``seed`` overrides the default seed (= k).
    """
    s = k if seed is None else seed
    if k == 1:
        return uniform_cloud(CONFIG_NAMES[1], 256, 256, 8e-6, 632.8e-9, n or 128,
                             1e-3, 0.1, 0.2, 0.0, 1.0, s)
    if k == 2:
        return uniform_cloud(CONFIG_NAMES[2], 1920, 1080, 8e-6, 532e-9, n or 10000,
                             3e-3, 0.5, 0.6, 0.0, 1.0, s)
    if k == 3:
        return uniform_cloud(CONFIG_NAMES[3], 2048, 2048, 8e-6, 532e-9, n or 65536,
                             4e-3, 0.4, 0.8, 0.0, 1.0, s)
    if k == 5:
        return ellipsoid_cloud(CONFIG_NAMES[5], 4096, 4096, 4e-6, 532e-9, n or 1_000_000,
                               seed=s)
    raise ValueError(f"no single-hologram configuration {k}")


# Wavefront-recording workload: a shallow object 5 mm deep, the virtual plane
# 5 mm in front of its nearest points (distances to the plane 5 .. 10 mm, disc
# radii 21 .. 42 samples), on a 2048 x 2048 plane holding the 1920 x 1080
# hologram centred.
WRM_PLANE_Z = 0.495
WRM_PLANE_N = 2048


def make_wrm(n: int = 10000, seed: int = 7) -> Cloud:
    """The wavefront-recording workload (Table 8's hologram: 1920 x 1080, 8 um;
    1e3 .. 1e5 points): x, y ~ U(+-3 mm), z ~ U[0.5, 0.505] m, A ~ U[0, 1],
    532 nm.  The virtual plane lies at WRM_PLANE_Z from the hologram."""
    c = uniform_cloud(f"W 1920x1080 p=8um 532nm N={n} z 0.5..0.505", 1920, 1080, 8e-6, 532e-9,
                      n, 3e-3, 0.5, 0.505, 0.0, 1.0, seed)
    c.meta["plane_z"] = WRM_PLANE_Z
    c.meta["plane_n"] = WRM_PLANE_N
    return c


def make_batch(n_frames: int = 64, width: int = 1920, height: int = 1080,
               n_lo: int = 1000, n_hi: int = 50000, seed_base: int = 400,
               counts: Optional[List[int]] = None) -> Batch:
    """Batch workload 4: frames of uneven point counts and cycled wavelengths.

    Frame f: seed = seed_base + f; N_f = round(exp(U[ln n_lo, ln n_hi])) drawn
    first, then x, y ~ U(-3 mm, 3 mm), z ~ U[0.3, 1.0] m, amplitude ~ U[0, 1].
    ``counts`` fixes the N_f instead (for reduced-size tests).
    """
    xs, ys, zs, as_, cnt, seeds = [], [], [], [], [], []
    for f in range(n_frames):
        s = seed_base + f
        rng = np.random.default_rng(s)
        nf = int(round(float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))))
        if counts is not None:
            nf = int(counts[f])
        xs.append(rng.uniform(-3e-3, 3e-3, nf))
        ys.append(rng.uniform(-3e-3, 3e-3, nf))
        zs.append(rng.uniform(0.3, 1.0, nf))
        as_.append(rng.uniform(0.0, 1.0, nf))
        cnt.append(nf)
        seeds.append(s)
    counts_a = np.asarray(cnt, dtype=np.int64)
    offsets = np.zeros(n_frames, dtype=np.int64)
    if n_frames > 1:
        offsets[1:] = np.cumsum(counts_a)[:-1]
    lam = np.asarray([BATCH_WAVELENGTHS[f % 3] for f in range(n_frames)], dtype=np.float64)
    cat = (lambda parts: np.concatenate(parts) if parts else np.zeros(0))
    return Batch(f"C4 {n_frames}x({width}x{height})", width, height, 8e-6,
                 _f32(cat(xs)), _f32(cat(ys)), _f32(cat(zs)), _f32(cat(as_)),
                 offsets, counts_a, lam, seeds)


def strided_pixels(width: int, height: int, step: int):
    """Every ``step``-th row and column, starting at 0 (corners' rows/cols included)."""
    ix = np.arange(0, width, step, dtype=np.int32)
    iy = np.arange(0, height, step, dtype=np.int32)
    return ix, iy


def crop_pixels(x0: int, y0: int, w: int, h: int):
    """Columns [x0, x0+w) and rows [y0, y0+h)."""
    return np.arange(x0, x0 + w, dtype=np.int32), np.arange(y0, y0 + h, dtype=np.int32)
