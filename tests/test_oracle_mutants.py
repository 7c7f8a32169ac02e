"""The oracle's pins catch plausible slips: each case plants one mistake in a
copy of the C oracle (a dropped term, a wrong sign or constant, a swapped
index, an off-by-half centre, a lost row), builds it, and runs every pin of
tests/test_oracle.py against it; likewise for the numpy Fourier form of
Eq. (10) (no padding, wrong offsets, wrong constant, wrong crop).  At least one pin must fail for every
mutant, and all pins must pass again on the real oracle afterwards.

CPU only; the mistakes are planted in the oracle, never in GPU code.
"""
import os
import shutil
import subprocess

import pytest

import oracle
import test_oracle as pins

# (name, exact text in cgh_oracle.c, replacement); each text occurs once
MUTANTS = [
    ("phase sign", "theta = pi * (dx * dx + dy * dy) / (jb->wavelength * jb->z[j]);",
     "theta = -pi * (dx * dx + dy * dy) / (jb->wavelength * jb->z[j]);"),
    ("phase factor 2", "theta = pi * (dx * dx + dy * dy) / (jb->wavelength * jb->z[j]);",
     "theta = 2.0 * pi * (dx * dx + dy * dy) / (jb->wavelength * jb->z[j]);"),
    ("depth dropped", "theta = pi * (dx * dx + dy * dy) / (jb->wavelength * jb->z[j]);",
     "theta = pi * (dx * dx + dy * dy) / (jb->wavelength);"),
    ("x centre off by half a pixel", "const double half_w = 0.5 * (double)(jb->width - 1);",
     "const double half_w = 0.5 * (double)(jb->width);"),
    ("x and y of the point swapped", "const double dx = xh - jb->x[j];",
     "const double dx = xh - jb->y[j];"),
    ("amplitude dropped", "re += jb->a[j] * cos(theta);", "re += cos(theta);"),
    ("imaginary part uses cos", "im += jb->a[j] * sin(theta);", "im += jb->a[j] * cos(theta);"),
    ("last point skipped", "for (int64_t j = 0; j < jb->n_points; ++j) {",
     "for (int64_t j = 0; j + 1 < jb->n_points; ++j) {"),
    ("a thread's last row lost",
     "jb->spherical = spherical;\n        jb->row_begin = n_rows * t / n_threads;\n"
     "        jb->row_end = n_rows * (t + 1) / n_threads;",
     "jb->spherical = spherical;\n        jb->row_begin = n_rows * t / n_threads;\n"
     "        jb->row_end = n_rows * (t + 1) / n_threads - (t + 1 == n_threads && n_rows > 1);"),
    ("spherical: z dropped from the distance",
     "sqrt(dx * dx + dy * dy + jb->z[j] * jb->z[j]);", "sqrt(dx * dx + dy * dy);"),
    ("spherical: 2 pi dropped", "theta = 2.0 * pi / jb->wavelength *",
     "theta = pi / jb->wavelength *"),
    ("diffraction: conjugated impulse response", "re += ur * hr - ui * hi;",
     "re += ur * hr + ui * hi;"),
    ("diffraction: sample area dropped",
     "const double s = jb->pitch * jb->pitch / (jb->wavelength * jb->z);",
     "const double s = 1.0 / (jb->wavelength * jb->z);"),
    ("diffraction: input transposed", "const double ur = jb->u_re[(int64_t)k * n + l];",
     "const double ur = jb->u_re[(int64_t)l * n + k];"),
    ("diffraction: chirp off by a factor 2",
     "const double q = jb->pitch * jb->pitch / (2.0 * jb->wavelength * jb->z);",
     "const double q = jb->pitch * jb->pitch / (jb->wavelength * jb->z);"),
    ("diffraction: prefactor without the -i", "const double pr = s * ei, pi_ = -s * er;",
     "const double pr = s * er, pi_ = s * ei;"),
    ("recording: region radius doubled",
     "const double rj = jb->wavelength * d / (2.0 * jb->pitch);",
     "const double rj = jb->wavelength * d / jb->pitch;"),
    ("recording: depth from the hologram, not the plane",
     "const double d = jb->z[i] - jb->zw;", "const double d = jb->z[i];"),
    ("recording: points in front of the plane recorded", "if (!(d > 0.0))\n                    continue;",
     "if (d == 0.0)\n                    continue;"),
    ("recording: phase sign", "const double theta = pi * rr / (jb->wavelength * d);",
     "const double theta = -pi * rr / (jb->wavelength * d);"),
    ("recording: centre off by half a sample", "const double half = 0.5 * (double)(jb->n - 1);",
     "const double half = 0.5 * (double)(jb->n);"),
    ("recording: x offset from the point's y", "const double dx = xw - jb->x[i];",
     "const double dx = xw - jb->y[i];"),
    ("recording: amplitude dropped", "sum_re += jb->a[i] * cos(theta);", "sum_re += cos(theta);"),
    ("recording: region not applied", "if (rr > rj * rj)\n                    continue;",
     "if (rr < 0.0)\n                    continue;"),
    ("recording: last point skipped", "for (int64_t i = 0; i < jb->n_points; ++i) {",
     "for (int64_t i = 0; i + 1 < jb->n_points; ++i) {"),
]


def _pin_calls():
    """Every pin of test_oracle.py as a zero-argument call."""
    calls = []
    for name in sorted(dir(pins)):
        fn = getattr(pins, name)
        if not (name.startswith("test_") and callable(fn)):
            continue
        if name == "test_diffraction_direct_sum_equals_fourier_form":
            for n in (5, 8):
                calls.append((f"{name}[{n}]", lambda fn=fn, n=n: fn(n)))
        else:
            calls.append((name, fn))
    return calls


def _use_library(src, lib):
    oracle._lib = None
    oracle._SRC, oracle._LIB = src, lib


def _failing_pins():
    failed = []
    for name, call in _pin_calls():
        try:
            call()
        except (AssertionError, ValueError, RuntimeError, FloatingPointError):
            failed.append(name)
    return failed


@pytest.mark.parametrize("name,text,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_every_planted_mistake_fails_a_pin(name, text, repl, tmp_path):
    with open(oracle._SRC) as f:
        src = f.read()
    assert src.count(text) == 1, f"mutation site of '{name}' not unique"
    mut_src = os.path.join(tmp_path, "cgh_oracle_mutant.c")
    mut_lib = os.path.join(tmp_path, "libcgh_oracle_mutant.so")
    with open(mut_src, "w") as f:
        f.write(src.replace(text, repl))
    subprocess.run(["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
                    "-shared", "-pthread", mut_src, "-o", mut_lib, "-lm"], check=True)
    real = (oracle._SRC, oracle._LIB)
    try:
        _use_library(mut_src, mut_lib)
        failed = _failing_pins()
    finally:
        _use_library(*real)
    assert failed, f"no pin fails with the planted mistake '{name}'"


# the oracle's Fourier form of Eq. (10) (numpy): (name, text, replacement)
FFT_MUTANTS = [
    ("no zero padding (circular wrap-around)", "m = 2 * n", "m = n"),
    ("offsets not circular", "d = np.where(d < n, d, d - m)", "d = d"),
    ("sample area dropped", "* pitch * pitch", "* 1.0"),
    ("prefactor without 1/i", "/ (1j * wavelength * z)", "/ (wavelength * z)"),
    ("crop from the wrong corner", "np.fft.ifft2(spec)[:n, :n]", "np.fft.ifft2(spec)[n:, n:]"),
]


@pytest.mark.parametrize("name,text,repl", FFT_MUTANTS, ids=[m[0] for m in FFT_MUTANTS])
def test_every_planted_mistake_in_the_fourier_form_fails_a_pin(name, text, repl):
    import inspect
    import numpy as np
    src = inspect.getsource(oracle.diffraction_fft)
    assert src.count(text) == 1, f"mutation site of '{name}' not unique"
    ns = {"np": np}
    exec(src.replace(text, repl), ns)
    real = oracle.diffraction_fft
    try:
        oracle.diffraction_fft = ns["diffraction_fft"]
        failed = _failing_pins()
    finally:
        oracle.diffraction_fft = real
    assert failed, f"no pin fails with the planted mistake '{name}'"


def test_pins_pass_on_the_real_oracle():
    assert _failing_pins() == []


def test_mutant_builds_leave_the_real_library_alone():
    assert shutil.which("gcc")
    lib = oracle._load()
    assert os.path.samefile(lib._name, oracle._LIB)
