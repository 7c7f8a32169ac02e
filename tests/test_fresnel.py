"""GPU parity of the Fresnel diffraction of a sampled field (Eq. (10),
cgh_fresnel_*) against the FP64 oracle.

Tolerance: NRMS <= 1e-5 of the complex field (FP32 transforms; the measured
error is ~1e-6).  Small fields are compared with the oracle's direct
summation; larger ones with its Fourier form, which the CPU tests pin to the
direct sum; the largest (n = 8192, padded transforms of 16384) with the closed
form of a field of a few samples, whose propagation is a sum of shifted
impulse responses.
"""
import numpy as np
import pytest

import oracle
import paper_1309_2734_amd as cgh

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print("[fresnel]", *a, flush=True)


def field(n, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)


def gpu(u, p, lam, z, plan=None, inplace=False):
    import torch
    n = u.shape[0]
    own = plan is None
    if own:
        plan = cgh.FresnelPlan(n, p, lam, z)
    ut = torch.from_numpy(np.ascontiguousarray(u)).cuda()
    out = ut if inplace else torch.empty_like(ut)
    plan.run(ut, out)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.complex128)
    if own:
        plan.close()
    return res


def nrms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n", [16, 32, 64])
def test_small_fields_match_direct_sum(n):
    u = field(n, n)
    for p, lam, z in ((8e-6, 532e-9, 0.02), (4e-6, 633e-9, -0.01)):
        ref = oracle.diffraction(u.astype(np.complex128), p, lam, z)
        got = gpu(u, p, lam, z)
        e = nrms(got, ref)
        say(f"n={n} z={z}: nrms {e:.3e}")
        assert np.all(np.isfinite(got))
        assert e <= TOL


@pytest.mark.parametrize("n", [128, 512, 2048])
def test_fields_match_fourier_form(n):
    u = field(n, 7 + n)
    p, lam, z = 8e-6, 532e-9, 0.05
    ref = oracle.diffraction_fft(u.astype(np.complex128), p, lam, z)
    got = gpu(u, p, lam, z)
    e = nrms(got, ref)
    say(f"n={n}: nrms {e:.3e}")
    assert e <= TOL


@pytest.mark.parametrize("n", [256, 2048])       # column passes; row passes and transposes
def test_in_place_and_repeated_runs(n):
    u = field(n, 3)
    p, lam, z = 6e-6, 473e-9, 0.03
    ref = oracle.diffraction_fft(u.astype(np.complex128), p, lam, z)
    plan = cgh.FresnelPlan(n, p, lam, z)
    a = gpu(u, p, lam, z, plan=plan)
    b = gpu(u, p, lam, z, plan=plan, inplace=True)
    plan.close()
    assert np.array_equal(a, b)
    assert nrms(a, ref) <= TOL


@pytest.mark.parametrize("n", [1024, 8192])
def test_few_samples_closed_form(n):
    """u = three samples: O = C p^2 sum_s a_s h(m - k_s, c - l_s), evaluated in
    FP64 on a set of rows (the corners of the grid included)."""
    p, lam, z = 4e-6, 532e-9, 0.5
    pts = [(0, 0, 1.0 + 0.0j), (n // 2 + 3, n // 3, -0.5 + 0.8j), (n - 1, n - 2, 0.3 - 0.1j)]
    u = np.zeros((n, n), dtype=np.complex64)
    for k, l, a in pts:
        u[k, l] = a
    got = gpu(u, p, lam, z)
    rows = np.array([0, 1, n // 2, n - 2, n - 1])
    c = np.arange(n, dtype=np.float64)[None, :]
    q = p * p / (2.0 * lam * z)
    want = np.zeros((rows.size, n), dtype=np.complex128)
    for k, l, a in pts:
        rev = np.fmod(q * ((rows[:, None] - k).astype(np.float64) ** 2 + (c - l) ** 2), 1.0)
        want += complex(a) * np.exp(2j * np.pi * rev)
    zrev = np.fmod(z / lam, 1.0)
    want *= np.exp(2j * np.pi * zrev) / (1j * lam * z) * p * p
    e = nrms(got[rows], want)
    say(f"n={n} few samples: nrms {e:.3e}")
    assert e <= TOL


def test_run_argument_checks():
    import torch
    plan = cgh.FresnelPlan(32, 8e-6, 532e-9, 0.02)
    with pytest.raises(TypeError):
        plan.run(torch.zeros((32, 32), device="cuda"), torch.zeros((32, 32), device="cuda"))
    with pytest.raises(TypeError):
        plan.run(torch.zeros((16, 16), dtype=torch.complex64, device="cuda"),
                 torch.zeros((16, 16), dtype=torch.complex64, device="cuda"))
    # through the C-ABI: a buffer off its 8-byte alignment is refused before
    # anything is launched
    buf = torch.zeros((33, 32), dtype=torch.complex64, device="cuda")
    assert cgh.lib().cgh_fresnel_run(plan._h, buf.data_ptr() + 4, buf.data_ptr(), None) == cgh.EINVAL
    assert cgh.lib().cgh_fresnel_run(plan._h, buf.data_ptr(), buf.data_ptr() + 4, None) == cgh.EINVAL
    torch.cuda.synchronize()
    plan.close()


@pytest.mark.parametrize("n", [512, 2048])
def test_graph_replays_match_eager(n):
    """A run captured into a HIP graph (torch's graph capture) replays the
    eager result bit for bit, with other eager diffraction work and
    synchronisations between the replays (both pipelines: column passes up
    to n = 1024, row passes and transposes above)."""
    import torch
    p, lam, z = 8e-6, 532e-9, 0.04
    u = torch.from_numpy(field(n, 11)).cuda()
    plan = cgh.FresnelPlan(n, p, lam, z)
    eager = torch.empty_like(u)
    plan.run(u, eager)
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    out = torch.empty_like(u)
    other = cgh.FresnelPlan(256, 4e-6, 633e-9, -0.02)
    v = torch.from_numpy(field(256, 12)).cuda()
    w = torch.empty_like(v)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        plan.run(u, out, torch.cuda.current_stream())        # warm-up on the side stream
        side.synchronize()
        with torch.cuda.graph(g, stream=side):
            plan.run(u, out, side)
    torch.cuda.synchronize()
    for rep in range(4):
        say(f"graph replay {rep}")
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), f"replay {rep}"
        other.run(v, w)                                   # eager work between replays
        torch.cuda.synchronize()
    del g
    plan.close()
    other.close()
