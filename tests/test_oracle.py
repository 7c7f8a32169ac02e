"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

The paper prints no hologram values, so the oracle is pinned by closed forms,
invariants, the paper's own recurrence relation (Section 2.2, Eq. (6)-(8))
evaluated in exact rational arithmetic, and 40-digit brute force.  Each pin
is chosen so that a plausible slip in the oracle (a dropped term, a wrong
constant or sign, a swapped x/y, an off-by-half pixel centre, a missed point)
fails at least one of them.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import cghgen
import oracle


# ---------------------------------------------------------------- Z1
def _zone_plate_setup():
    # beta = p^2 / (2 lambda z) = 1/8 revolution per pixel^2, so that the
    # phase at integer pixel offsets (n, m) from the point is (n^2 + m^2)/8
    # revolutions and I takes the exact values cos(pi k / 4).
    p = 8e-6
    z = 2.0 ** -11            # exactly representable
    lam = 4.0 * p * p / z     # 524.288 nm
    return p, z, lam


def test_z1_zone_plate_closed_form():
    """Single off-centre point on an odd, non-square grid: Eq. (2) gives
    I = cos(2 pi beta ((ix-ix0)^2 + (iy-iy0)^2)) exactly (pins pi/(lambda z),
    the pixel-centre convention and x/y orientation)."""
    W, H = 255, 129
    p, z, lam = _zone_plate_setup()
    ix0, iy0 = 127 + 3, 64 - 5            # pixel (W-1)/2 + 3, (H-1)/2 - 5
    x = [3 * p]
    y = [-5 * p]
    re, im = oracle.fresnel_complex(W, H, p, lam, x, y, [z], [1.0], threads=4)
    n = np.arange(W)[None, :] - ix0
    m = np.arange(H)[:, None] - iy0
    k = (n * n + m * m) % 8
    exp_re = np.cos(np.pi * k / 4.0)
    exp_im = np.sin(np.pi * k / 4.0)
    assert np.max(np.abs(re - exp_re)) < 1e-9
    # the imaginary part pins the sign convention exp(+i phase) of Eq. (2)
    assert np.max(np.abs(im - exp_im)) < 1e-9


def test_z1_amplitude_scales_zone_plate():
    W, H = 63, 31
    p, z, lam = _zone_plate_setup()
    I = oracle.fresnel(W, H, p, lam, [0.0], [0.0], [z], [0.375])
    n = np.arange(W)[None, :] - 31
    m = np.arange(H)[:, None] - 15
    exp = 0.375 * np.cos(np.pi * ((n * n + m * m) % 8) / 4.0)
    assert np.max(np.abs(I - exp)) < 1e-10


def test_z1_kinoform_codes_of_zone_plate():
    """Eq. (3) on the zone plate: theta = pi k / 4, code = floor(k * 255 / 8).
    For k != 0 no code is near a quantisation boundary; k = 0 sits on the
    0 / 2 pi wrap, where rounding of Im O decides between 0 and the top codes
    (254, or 255 when the FP32 wrap rounds theta up to 2 pi)."""
    W, H = 45, 33
    p, z, lam = _zone_plate_setup()
    re, im = oracle.fresnel_complex(W, H, p, lam, [0.0], [0.0], [z], [1.0])
    codes = oracle.kinoform(re, im)
    n = np.arange(W)[None, :] - 22
    m = np.arange(H)[:, None] - 16
    k = (n * n + m * m) % 8
    exp = (k * 255) // 8
    got = codes.astype(np.int64)
    assert np.array_equal(got[k != 0], exp[k != 0])
    assert np.all(np.isin(got[k == 0], [0, 254, 255]))


# ---------------------------------------------------------------- Z2
def test_z2_linearity_in_amplitude():
    c = cghgen.make_config(1, n=40)
    rng = np.random.default_rng(11)
    A = rng.uniform(0, 1, c.n)
    B = rng.uniform(-1, 1, c.n)
    al, be = 0.7, -1.3
    args = (c.width, c.height, c.pitch, c.wavelength, c.x, c.y, c.z)
    IA = oracle.fresnel(*args, A, rows=range(0, 256, 5))
    IB = oracle.fresnel(*args, B, rows=range(0, 256, 5))
    IAB = oracle.fresnel(*args, al * A + be * B, rows=range(0, 256, 5))
    scale = np.max(np.abs(IAB))
    assert np.max(np.abs(IAB - (al * IA + be * IB))) < 1e-12 * max(scale, 1.0) * c.n


def test_z2_zero_amplitude_and_empty_cloud():
    c = cghgen.make_config(1, n=16)
    args = (c.width, c.height, c.pitch, c.wavelength)
    assert np.all(oracle.fresnel(*args, c.x, c.y, c.z, np.zeros(c.n)) == 0.0)
    empty = np.zeros(0)
    I0 = oracle.fresnel(*args, empty, empty, empty, empty)
    assert I0.shape == (c.height, c.width) and np.all(I0 == 0.0)


def test_superposition_over_point_sets():
    """I(P1 u P2) = I(P1) + I(P2): every point contributes once."""
    c = cghgen.make_config(1, n=33)
    args = (c.width, c.height, c.pitch, c.wavelength)
    sl1, sl2 = slice(0, 20), slice(20, 33)
    rows = range(0, 256, 7)
    I = oracle.fresnel(*args, c.x, c.y, c.z, c.amp, rows=rows)
    I1 = oracle.fresnel(*args, c.x[sl1], c.y[sl1], c.z[sl1], c.amp[sl1], rows=rows)
    I2 = oracle.fresnel(*args, c.x[sl2], c.y[sl2], c.z[sl2], c.amp[sl2], rows=rows)
    assert np.max(np.abs(I - (I1 + I2))) < 1e-12 * c.n
    # each single point alone has |I| <= A_j, with equality on its own zone centre
    Ij = oracle.fresnel(*args, c.x[:1], c.y[:1], c.z[:1], c.amp[:1], rows=rows)
    assert np.max(np.abs(Ij)) <= float(c.amp[0]) * (1 + 1e-15)


# ---------------------------------------------------------------- Z3
def test_z3_mirror_symmetry_bitwise():
    c = cghgen.make_config(1, n=24)
    args = (c.width, c.height, c.pitch, c.wavelength)
    I = oracle.fresnel(*args, c.x, c.y, c.z, c.amp)
    Ix = oracle.fresnel(*args, -c.x.astype(np.float64), c.y, c.z, c.amp)
    Iy = oracle.fresnel(*args, c.x, -c.y.astype(np.float64), c.z, c.amp)
    assert np.array_equal(Ix, I[:, ::-1])
    assert np.array_equal(Iy, I[::-1, :])
    # square grid: swapping the roles of x and y transposes the hologram
    It = oracle.fresnel(*args, c.y, c.x, c.z, c.amp)
    assert np.array_equal(It, I.T)


def test_z3_mirror_nonsquare_even_odd():
    c = cghgen.make_config(1, n=9)
    for W, H in ((64, 37), (33, 16)):
        I = oracle.fresnel(W, H, c.pitch, c.wavelength, c.x, c.y, c.z, c.amp)
        Ix = oracle.fresnel(W, H, c.pitch, c.wavelength, -c.x.astype(np.float64), c.y, c.z, c.amp)
        assert np.array_equal(Ix, I[:, ::-1])


# ---------------------------------------------------------------- Z4
def test_z4_integer_pixel_translation():
    c = cghgen.make_config(1, n=20)
    k, l = 5, -3
    x2 = c.x.astype(np.float64) + k * c.pitch
    y2 = c.y.astype(np.float64) + l * c.pitch
    args = (c.width, c.height, c.pitch, c.wavelength)
    I = oracle.fresnel(*args, c.x, c.y, c.z, c.amp)
    I2 = oracle.fresnel(*args, x2, y2, c.z, c.amp)
    # I2[iy + l, ix + k] == I[iy, ix] on the overlap
    a = I2[max(l, 0):c.height + min(l, 0), max(k, 0):c.width + min(k, 0)]
    b = I[max(-l, 0):c.height + min(-l, 0), max(-k, 0):c.width + min(-k, 0)]
    assert a.shape == b.shape and a.size > 0
    assert np.max(np.abs(a - b)) < 1e-10 * max(1.0, np.max(np.abs(b)))


# ---------------------------------------------------------------- Z5
def test_z5_separable_complex_matrix_product():
    """Re(Y diag(A) X^T) with numpy's complex128 matrix product equals the
    direct sum (the factorisation of exp(i(a+b)) = exp(ia) exp(ib))."""
    c = cghgen.make_config(1)
    x = c.x.astype(np.float64); y = c.y.astype(np.float64)
    z = c.z.astype(np.float64); A = c.amp.astype(np.float64)
    xh = (np.arange(c.width) - (c.width - 1) / 2.0) * c.pitch
    yh = (np.arange(c.height) - (c.height - 1) / 2.0) * c.pitch
    X = np.exp(1j * np.pi * (xh[:, None] - x[None, :]) ** 2 / (c.wavelength * z[None, :]))
    Y = np.exp(1j * np.pi * (yh[:, None] - y[None, :]) ** 2 / (c.wavelength * z[None, :]))
    ref = np.real((Y * A[None, :]) @ X.T)
    I = oracle.cloud_fresnel(c)
    assert np.max(np.abs(I - ref)) < 1e-10 * np.sqrt(np.mean(ref ** 2)) * 10


# ---------------------------------------------------------------- Z6
def _mp_hologram(width, height, pitch, lam, x, y, z, a, cols, rows, spherical=False):
    with mpmath.workdps(40):
        P = mpmath.mpf(pitch); L = mpmath.mpf(lam)
        hw = mpmath.mpf(width - 1) / 2; hh = mpmath.mpf(height - 1) / 2
        re = np.zeros((len(rows), len(cols))); im = np.zeros_like(re)
        for r, iy in enumerate(rows):
            yh = (iy - hh) * P
            for cc, ix in enumerate(cols):
                xh = (ix - hw) * P
                sr = mpmath.mpf(0); si = mpmath.mpf(0)
                for j in range(len(x)):
                    dx = xh - mpmath.mpf(float(x[j])); dy = yh - mpmath.mpf(float(y[j]))
                    zj = mpmath.mpf(float(z[j]))
                    if spherical:
                        th = 2 * mpmath.pi / L * mpmath.sqrt(dx * dx + dy * dy + zj * zj)
                    else:
                        th = mpmath.pi * (dx * dx + dy * dy) / (L * zj)
                    sr += mpmath.mpf(float(a[j])) * mpmath.cos(th)
                    si += mpmath.mpf(float(a[j])) * mpmath.sin(th)
                re[r, cc] = float(sr); im[r, cc] = float(si)
    return re, im


def test_z6_brute_force_40_digits_corner_of_c2():
    c = cghgen.make_config(2, n=3)
    cols = [0, 1, 1918, 1919]
    rows = [0, 540, 1079]
    ref_re, ref_im = _mp_hologram(c.width, c.height, c.pitch, c.wavelength, c.x, c.y, c.z,
                                  c.amp, cols, rows)
    re, im = oracle.fresnel_complex(c.width, c.height, c.pitch, c.wavelength, c.x, c.y, c.z,
                                    c.amp, cols=cols, rows=rows)
    assert np.max(np.abs(re - ref_re)) < 1e-11
    assert np.max(np.abs(im - ref_im)) < 1e-11


def test_z6_brute_force_spherical_eq1():
    c = cghgen.make_config(1, n=3)
    cols = [0, 100, 255]
    rows = [0, 128, 255]
    ref_re, ref_im = _mp_hologram(c.width, c.height, c.pitch, c.wavelength, c.x, c.y, c.z,
                                  c.amp, cols, rows, spherical=True)
    re, im = oracle.spherical_complex(c.width, c.height, c.pitch, c.wavelength, c.x, c.y,
                                      c.z, c.amp, cols=cols, rows=rows)
    # phase ~ 2 pi z / lambda ~ 2e6 rad: FP64 keeps it to ~1e-9 rad
    assert np.max(np.abs(re - ref_re)) < 1e-8
    assert np.max(np.abs(im - ref_im)) < 1e-8


def test_spherical_approaches_fresnel_plus_depth_term():
    """Eq. (1) vs Eq. (2): the exact phase exceeds the Fresnel phase (with its
    2 pi z_j / lambda term) by 2 pi/lambda * (-r^4 / (8 z^3) + ...), so for a
    point far away the two agree to that bound."""
    p, lam, z = 8e-6, 532e-9, 2.0
    W = H = 17
    x, y = [1e-5], [-2e-5]
    re_s, im_s = oracle.spherical_complex(W, H, p, lam, x, y, [z], [1.0])
    re_f, im_f = oracle.fresnel_complex(W, H, p, lam, x, y, [z], [1.0])
    # Fresnel with the depth term: multiply by exp(i 2 pi z / lambda), taken exactly
    with mpmath.workdps(30):
        ph = float(mpmath.fmod(2 * mpmath.pi * mpmath.mpf(z) / mpmath.mpf(lam), 2 * mpmath.pi))
    o_f = (re_f + 1j * im_f) * np.exp(1j * ph)
    r2 = ((np.arange(W)[None, :] - 8) * p - x[0]) ** 2 + ((np.arange(H)[:, None] - 8) * p - y[0]) ** 2
    bound = 2 * np.pi / lam * r2 ** 2 / (8 * z ** 3)
    diff = np.abs((re_s + 1j * im_s) - o_f)
    assert np.all(diff <= 1.01 * bound + 1e-7)


# ---------------------------------------------------------------- Z7
def test_z7_recurrence_relation_eq6_to_8():
    """The paper's recurrence (Eq. (6)-(8)) in exact rational arithmetic, with
    P_j = p^2 / (2 lambda z_j) for pixel-unit offsets: Gamma_1 is the phase at
    the row's first pixel, Gamma_{n+1} = Gamma_n + delta_n, delta_{n+1} =
    delta_n + 2 P_j.  cos(2 pi Gamma_{n+1}) must equal the oracle at pixel n."""
    c = cghgen.make_config(2, n=1)
    W, H = 96, 7
    row = 3
    p = Fraction(c.pitch); lam = Fraction(c.wavelength)
    xj = Fraction(float(c.x[0])); yj = Fraction(float(c.y[0])); zj = Fraction(float(c.z[0]))
    P = p * p / (2 * lam * zj)
    dx = (Fraction(0) - Fraction(W - 1, 2)) - xj / p     # pixel units
    dy = (Fraction(row) - Fraction(H - 1, 2)) - yj / p
    gamma = P * (dx * dx + dy * dy)
    delta = P * (2 * dx + 1)
    big_delta = 2 * P
    expect = []
    for n in range(W):
        frac = gamma - math.floor(gamma)
        with mpmath.workdps(30):
            expect.append(float(mpmath.cospi(2 * mpmath.mpf(frac.numerator) / frac.denominator)))
        gamma, delta = gamma + delta, delta + big_delta
    I = oracle.fresnel(W, H, c.pitch, c.wavelength, c.x, c.y, c.z, [1.0], rows=[row])
    assert np.max(np.abs(I[0] - np.asarray(expect))) < 1e-11


# ---------------------------------------------------------------- Z8 and plumbing
def test_z8_mean_energy_loose():
    c = cghgen.make_config(1)
    I = oracle.cloud_fresnel(c)
    e = float(np.mean(I * I))
    expect = float(np.sum(c.amp.astype(np.float64) ** 2) / 2)
    assert 0.5 * expect < e < 2.0 * expect


def test_subset_and_thread_count_are_bitwise_consistent():
    c = cghgen.make_config(1, n=50)
    full = oracle.cloud_fresnel(c, threads=1)
    cols = [0, 7, 128, 255]
    rows = [255, 3, 100]
    sub = oracle.cloud_fresnel(c, cols=cols, rows=rows, threads=3)
    assert np.array_equal(sub, full[np.ix_(rows, cols)])
    assert np.array_equal(oracle.cloud_fresnel(c, threads=8), full)


def test_oracle_rejects_bad_arguments():
    with pytest.raises(RuntimeError):
        oracle.fresnel(0, 4, 8e-6, 5e-7, [0.0], [0.0], [0.1], [1.0])
    with pytest.raises(RuntimeError):
        oracle.fresnel(4, 4, -8e-6, 5e-7, [0.0], [0.0], [0.1], [1.0])
    with pytest.raises(ValueError):
        oracle.fresnel(4, 4, 8e-6, 5e-7, [0.0, 1.0], [0.0], [0.1], [1.0])


def test_nrms_and_max_err_definitions():
    ref = np.array([3.0, -4.0])
    assert oracle.nrms(ref, ref) == 0.0
    assert abs(oracle.nrms(ref + np.array([0.3, 0.4]), ref) - 0.1) < 1e-15
    assert abs(oracle.max_err(ref + np.array([0.0, 0.5]), ref) - 0.5 / math.sqrt(12.5)) < 1e-15


# ---------------------------------------------------------------- Eq. (10)
# Fresnel diffraction of a sampled field (Section 2.3): direct summation and
# the Fourier form of the same equation.
def _field(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


def test_diffraction_of_one_sample_is_the_scaled_impulse_response():
    """u = a at (k0, l0), zero elsewhere: Eq. (10) reduces to the prefactor
    exp(i 2 pi z / lambda) / (i lambda z) p^2 times a exp(i pi p^2 ((m-k0)^2 +
    (c-l0)^2) / (lambda z)) at every output sample."""
    n, k0, l0, a = 12, 3, 8, 0.7 - 0.2j
    p, lam, z = 10e-6, 633e-9, 0.03
    u = np.zeros((n, n), dtype=np.complex128)
    u[k0, l0] = a
    got = oracle.diffraction(u, p, lam, z)
    m = np.arange(n)[:, None]
    c = np.arange(n)[None, :]
    h = np.exp(1j * np.pi * p * p * ((m - k0) ** 2 + (c - l0) ** 2) / (lam * z))
    # z / lambda is ~47,000 revolutions: its phase is taken to 40 digits
    with mpmath.workdps(40):
        ph = mpmath.mpf(2) * mpmath.pi * mpmath.mpf(z) / mpmath.mpf(lam)
        e = complex(mpmath.cos(ph), mpmath.sin(ph))
    pref = e / (1j * lam * z) * p * p
    want = pref * a * h
    # the oracle's FP64 z / lambda carries ~4e-12 revolution of rounding
    tol = 1e-10 * np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= tol
    # and the Fourier form agrees
    assert np.max(np.abs(oracle.diffraction_fft(u, p, lam, z) - want)) <= tol


@pytest.mark.parametrize("n", [5, 8, 16, 33])
def test_diffraction_direct_sum_equals_fourier_form(n):
    """The two lines of Eq. (10): the direct sum and F^-1[F[u] F[h]] on the
    2n-padded grid, cropped, agree to rounding for any field (odd n too)."""
    u = _field(n, n)
    for p, lam, z in ((8e-6, 532e-9, 0.02), (4e-6, 473e-9, -0.05)):
        a = oracle.diffraction(u, p, lam, z)
        b = oracle.diffraction_fft(u, p, lam, z)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_diffraction_conjugate_and_linearity():
    """Propagating conj(u) by -z gives conj of propagating u by z (h and the
    prefactor conjugate with z); the map is linear."""
    n, p, lam, z = 10, 8e-6, 532e-9, 0.015
    u, v = _field(n, 1), _field(n, 2)
    a = oracle.diffraction(u, p, lam, z)
    assert np.max(np.abs(oracle.diffraction(np.conj(u), p, lam, -z) - np.conj(a))) <= 1e-12 * np.max(np.abs(a))
    b = oracle.diffraction(v, p, lam, z)
    ab = oracle.diffraction(2.0 * u - 0.5j * v, p, lam, z)
    assert np.max(np.abs(ab - (2.0 * a - 0.5j * b))) <= 1e-12 * np.max(np.abs(ab))


def test_diffraction_row_subset_is_consistent():
    n = 16
    u = _field(n, 3)
    full = oracle.diffraction(u, 8e-6, 532e-9, 0.02, threads=1)
    sub = oracle.diffraction(u, 8e-6, 532e-9, 0.02, rows=[15, 0, 7], threads=3)
    assert np.array_equal(sub, full[[15, 0, 7]])


# -------------------------------------- wavefront recording, first step
def _wrm_closed_form_setup():
    # p = 2^-17 m, d = 2^-11 m, lambda = 5 * 2^-23 m (all exact): beta =
    # p^2 / (2 lambda d) = 1/10 revolution per sample^2 and the region radius
    # lambda d / (2 p) = 2.5 samples, so the disc holds the offsets with
    # k^2 + l^2 <= 6 (squared radius 6.25 is no sum of two squares: no ties).
    p = 2.0 ** -17
    d = 2.0 ** -11
    lam = 5.0 * 2.0 ** -23
    zw = 2.0 ** -10
    return p, d, lam, zw


def test_wrm_one_point_closed_form():
    """One point at sample (m, c) = (5, 9) of a 16 x 16 plane (x_j = 1.5 p,
    y_j = -2.5 p from the centre 7.5), d = z_j - zw = 2^-11 m beyond the
    plane: the recorded wave is exp(i pi s / 5) at the 21 samples of squared
    offset s in {0, 1, 2, 4, 5} and zero everywhere else.  The values are
    the exact algebraic cos / sin of multiples of pi / 5.  A second point in
    front of the plane (d < 0) and a third whose disc lies outside the plane
    add nothing.  Pins the region radius lambda d / (2 p), the distance
    d = z - zw, the phase scaling pi / (lambda d), the centre convention and
    the sign of the exponent."""
    p, d, lam, zw = _wrm_closed_form_setup()
    x = [1.5 * p, 1.5 * p, 40.0 * p]
    y = [-2.5 * p, -2.5 * p, 40.0 * p]
    z = [zw + d, zw - d, zw + d]
    u = oracle.wrm_record(16, p, lam, zw, x, y, z, [1.0, 0.5, 1.0], threads=3)
    r5 = math.sqrt(5.0)
    cos_k = {0: 1.0, 1: (1 + r5) / 4, 2: (r5 - 1) / 4, 4: -(1 + r5) / 4, 5: -1.0}
    sin_k = {0: 0.0, 1: math.sqrt(10 - 2 * r5) / 4, 2: math.sqrt(10 + 2 * r5) / 4,
             4: math.sqrt(10 - 2 * r5) / 4, 5: 0.0}
    exp = np.zeros((16, 16), dtype=np.complex128)
    for m in range(16):
        for c in range(16):
            s = (m - 5) ** 2 + (c - 9) ** 2
            if s in cos_k:
                exp[m, c] = cos_k[s] + 1j * sin_k[s]
    assert np.count_nonzero(exp) == 21
    assert np.max(np.abs(u - exp)) < 1e-12


def test_wrm_equals_direct_sum_where_regions_cover_the_plane():
    """With every disc larger than the plane's diagonal the recorded plane is
    the unrestricted Fresnel sum of Eq. (2) at the depths d_j = z_j - zw: the
    direct-calculation oracle (pinned above) on the n x n grid."""
    n, p, lam, zw = 12, 8e-6, 532e-9, 0.05
    rng = np.random.default_rng(11)
    N = 9
    x = rng.uniform(-3 * p, 3 * p, N).astype(np.float32)
    y = rng.uniform(-3 * p, 3 * p, N).astype(np.float32)
    dmin = 2.0 * p * 40 * p / lam        # radius >= 40 p > the diagonal 12 sqrt(2) p
    d = rng.uniform(dmin, 2 * dmin, N)
    z = (zw + d).astype(np.float32)
    a = rng.uniform(0.2, 1.0, N).astype(np.float32)
    u = oracle.wrm_record(n, p, lam, zw, x, y, z, a)
    dd = z.astype(np.float64) - zw           # the same FP64 depths
    re, im = oracle.fresnel_complex(n, n, p, lam, x, y, dd, a)
    assert np.max(np.abs(u - (re + 1j * im))) < 1e-12


def test_wrm_superposition_mirror_and_rows():
    """Partial discs: the plane of two point sets is the sum of their planes;
    mirroring x_j mirrors the columns bit for bit (centred grid); a row
    subset gives the same rows bit for bit."""
    n, p, lam, zw = 40, 8e-6, 532e-9, 0.4
    rng = np.random.default_rng(12)
    N = 14
    x = rng.uniform(-18 * p, 18 * p, N).astype(np.float32)
    y = rng.uniform(-18 * p, 18 * p, N).astype(np.float32)
    z = (zw + rng.uniform(0.0005, 0.0015, N)).astype(np.float32)   # radii 2 .. 6 samples
    a = rng.uniform(0.2, 1.0, N).astype(np.float32)
    full = oracle.wrm_record(n, p, lam, zw, x, y, z, a)
    parts = (oracle.wrm_record(n, p, lam, zw, x[:6], y[:6], z[:6], a[:6]) +
             oracle.wrm_record(n, p, lam, zw, x[6:], y[6:], z[6:], a[6:]))
    assert np.max(np.abs(full - parts)) < 1e-12
    mir = oracle.wrm_record(n, p, lam, zw, -x, y, z, a)
    assert np.array_equal(mir[:, ::-1], full)
    rows = [0, 7, 19, 39]
    assert np.array_equal(oracle.wrm_record(n, p, lam, zw, x, y, z, a, rows=rows, threads=2),
                          full[rows])
    # some discs are clipped by the plane's edge, some samples are outside all
    assert 0 < np.count_nonzero(full) < n * n
