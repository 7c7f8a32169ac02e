"""The seeded synthetic workloads: determinism, shapes and distributions."""
import numpy as np
import pytest

import cghgen


def test_same_seed_same_bytes():
    a = cghgen.make_config(2, n=500)
    b = cghgen.make_config(2, n=500)
    for f in ("x", "y", "z", "amp"):
        assert getattr(a, f).tobytes() == getattr(b, f).tobytes()
        assert getattr(a, f).dtype == np.float32
    c = cghgen.make_config(2, n=500, seed=99)
    assert c.x.tobytes() != a.x.tobytes()


@pytest.mark.parametrize("k,W,H,p,lam,n,xy,zlo,zhi", [
    (1, 256, 256, 8e-6, 632.8e-9, 128, 1e-3, 0.1, 0.2),
    (2, 1920, 1080, 8e-6, 532e-9, 10000, 3e-3, 0.5, 0.6),
    (3, 2048, 2048, 8e-6, 532e-9, 65536, 4e-3, 0.4, 0.8),
])
def test_uniform_configs(k, W, H, p, lam, n, xy, zlo, zhi):
    c = cghgen.make_config(k)
    assert (c.width, c.height, c.n) == (W, H, n)
    assert c.pitch == p and c.wavelength == lam
    assert np.all(np.abs(c.x) <= xy) and np.all(np.abs(c.y) <= xy)
    assert np.all(c.z >= np.float32(zlo)) and np.all(c.z <= np.float32(zhi))
    assert np.all(c.amp >= 0) and np.all(c.amp <= 1)
    # uniform: mean and spread close to the distribution's
    assert abs(float(np.mean(c.x))) < 4 * xy / np.sqrt(3 * n)
    assert abs(float(np.std(c.x.astype(np.float64))) - xy / np.sqrt(3)) < 0.05 * xy


def test_ellipsoid_surface_and_rotation():
    c = cghgen.make_config(5, n=20000)
    assert (c.width, c.height, c.pitch) == (4096, 4096, 4e-6)
    pts = np.stack([c.x, c.y, c.z], 1).astype(np.float64) - np.array([0, 0, 0.5])
    # rotation invariants: the ellipsoid's inertia eigen-axes are the semi-axes
    ev = np.sort(np.linalg.eigvalsh(pts.T @ pts / len(pts)))
    assert ev[-1] > ev[1] > ev[0]
    # every point is on the surface: after rotating back, sum (u_i/a_i)^2 = 1
    q = c.meta["rotation"]
    assert np.allclose(q @ q.T, np.eye(3), atol=1e-12)
    u = pts @ q                      # back to the ellipsoid's own frame
    r = np.sum((u / np.array([3e-3, 2e-3, 1e-3])) ** 2, axis=1)
    assert np.max(np.abs(r - 1.0)) < 1e-3   # float32 storage of z ~ 0.5 m
    # area-uniform, not angle-uniform: the flat faces (|u_z| small relative to
    # the sphere case) carry more points per solid angle
    assert abs(float(np.mean(u[:, 0] > 0)) - 0.5) < 0.02
    assert np.all(c.amp >= 0.5) and np.all(c.amp <= 1.0)


def test_batch_frames():
    b = cghgen.make_batch()
    assert b.n_frames == 64
    assert np.all(b.counts >= 1000) and np.all(b.counts <= 50000)
    assert np.array_equal(b.offsets[1:], np.cumsum(b.counts)[:-1]) and b.offsets[0] == 0
    assert b.x.shape[0] == int(b.counts.sum())
    assert list(b.wavelengths[:4]) == [633e-9, 532e-9, 473e-9, 633e-9]
    # log-uniform: mean of log N_f near the middle of [ln 1e3, ln 5e4]
    ml = float(np.mean(np.log(b.counts)))
    assert abs(ml - 0.5 * (np.log(1e3) + np.log(5e4))) < 0.6
    f = b.frame(5)
    assert f.n == b.counts[5] and f.wavelength == b.wavelengths[5]
    assert np.all(f.z >= np.float32(0.3)) and np.all(f.z <= np.float32(1.0))
    # frames are reproducible one by one
    b2 = cghgen.make_batch(n_frames=6)
    assert b2.frame(5).x.tobytes() == f.x.tobytes()


def test_batch_fixed_counts():
    b = cghgen.make_batch(n_frames=3, counts=[0, 5, 7])
    assert list(b.counts) == [0, 5, 7] and list(b.offsets) == [0, 0, 5]
