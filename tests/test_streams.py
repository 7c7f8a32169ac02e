"""Stream behaviour of the C-ABI calls (include/cgh.h, "Threads and streams").

- Compute calls only enqueue work: a call made while a long evaluation is
  still running returns before that evaluation ends, also when it needs new
  descriptor tables (another point chunking, another batch frame table),
  and every result equals the one computed with the host waiting in between.
- Calls on one context made on different streams are ordered by the library
  (they share its workspace): the second waits for the first.
- A captured batch graph reads only the batch's own tables: single-hologram
  calls on the same context between replays leave the replays unchanged.
"""
import numpy as np
import pytest

import cghgen
import oracle
import paper_1309_2734_amd as cgh

pytestmark = pytest.mark.gpu


def say(*a):
    print("[streams]", *a, flush=True)


def _host(t):
    return t.cpu().numpy().astype(np.float64)


def test_compute_calls_only_enqueue(monkeypatch):
    """2048 x 2048 hologram of 65,536 points in the direct FP32 mode (~30 ms
    of kernel time), then on the same stream: the split-BF16 hologram in
    point chunks of a small workspace, and a batch whose frame table differs
    from the previous batch's.  Both calls must return while the first
    evaluation still runs (the stream is not idle), and every output equals
    the one of a run with the host synchronised after each call."""
    import torch
    c = cghgen.make_config(3)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    shape = (c.height, c.width)
    long_ref, long_out = (torch.empty(shape, device="cuda") for _ in range(2))
    chunk_ref, chunk_out = (torch.empty(shape, device="cuda") for _ in range(2))
    frames_a = [(0, 4000, 633e-9), (5000, 3000, 532e-9), (9000, 2000, 473e-9)]
    frames_b = [(100, 1500, 532e-9), (7000, 2500, 633e-9)]
    batch_ref = torch.empty((len(frames_b),) + shape, device="cuda")
    batch_out = torch.empty_like(batch_ref)
    batch_a = torch.empty((len(frames_a),) + shape, device="cuda")
    s = torch.cuda.Stream()
    small = str(64 << 20)

    # reference pass, host waiting after every call; also grows every
    # workspace buffer the timed pass needs
    say("reference pass")
    ctx.compute(long_ref, cgh.DIRECT_FP32, stream=s)
    s.synchronize()
    monkeypatch.setenv("CGH_WORKSPACE_BYTES", small)
    ctx.compute(chunk_ref, cgh.SPLIT_BF16, stream=s)
    s.synchronize()
    monkeypatch.delenv("CGH_WORKSPACE_BYTES")
    ctx.batch_compute(frames_b, batch_ref, cgh.SPLIT_FP16, stream=s)
    s.synchronize()
    ctx.batch_compute(frames_a, batch_a, cgh.SPLIT_FP16, stream=s)   # a different table
    s.synchronize()

    say("timed pass")
    ctx.compute(long_out, cgh.DIRECT_FP32, stream=s)
    monkeypatch.setenv("CGH_WORKSPACE_BYTES", small)
    ctx.compute(chunk_out, cgh.SPLIT_BF16, stream=s)
    monkeypatch.delenv("CGH_WORKSPACE_BYTES")
    ctx.batch_compute(frames_b, batch_out, cgh.SPLIT_FP16, stream=s)
    busy = not s.query()
    s.synchronize()
    assert busy, "the calls did not return before the first evaluation ended"
    assert torch.equal(long_out, long_ref)
    assert torch.equal(chunk_out, chunk_ref)
    assert torch.equal(batch_out, batch_ref)
    # and the reference itself against the oracle on a few pixels
    cols, rows = np.arange(3, c.width, 257), np.arange(5, c.height, 263)
    ref = oracle.cloud_fresnel(c, cols=cols, rows=rows)
    for name, t, tol in (("direct", long_ref, 1e-5), ("split chunked", chunk_ref, 1e-3)):
        e = oracle.nrms(_host(t)[np.ix_(rows, cols)], ref)
        say(f"{name}: nrms {e:.3e}")
        assert e <= tol
    ctx.close()


def test_calls_on_two_streams_are_ordered():
    """A long direct evaluation on stream A, then the exact spherical wave on
    stream B: the second rewrites the constants and tables the first reads,
    so it must wait for it.  Both results equal their stand-alone results."""
    import torch
    c = cghgen.make_config(3)
    ctx = cgh.Context(c.width, c.height, c.pitch, c.wavelength)
    ctx.upload_cloud(c)
    shape = (c.height, c.width)
    a_ref, b_ref, a_out, b_out = (torch.empty(shape, device="cuda") for _ in range(4))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    say("stand-alone runs")
    ctx.compute(a_ref, cgh.DIRECT_FP32, stream=sa)
    sa.synchronize()
    ctx.compute(b_ref, cgh.SPHERICAL_FP32, stream=sb)
    sb.synchronize()
    for rep in range(2):
        say(f"two streams, round {rep}")
        ctx.compute(a_out, cgh.DIRECT_FP32, stream=sa)
        ctx.compute(b_out, cgh.SPHERICAL_FP32, stream=sb)
        sb.synchronize()
        sa.synchronize()
        assert torch.equal(a_out, a_ref)
        assert torch.equal(b_out, b_ref)
    ctx.close()


_MODES = (cgh.SPLIT_FP16, cgh.SPLIT_BF16, cgh.DIRECT_FP32, cgh.SEPARABLE_FP32)


@pytest.mark.parametrize("mode", _MODES, ids=lambda m: {v: k for k, v in cgh.MODES.items()}[m])
def test_batch_replays_after_single_calls_on_the_same_context(mode):
    """Replays of a captured batch graph, with single-hologram evaluations
    (real, complex, kinoform) and a tuning run on the same context in
    between, equal the eager batch bit for bit."""
    import torch
    counts = [0, 1, 37, 500, 2000, 33, 700]
    b = cghgen.make_batch(n_frames=len(counts), width=200, height=120, counts=counts)
    frames = cgh.batch_frames(b)
    ctx = cgh.Context(b.width, b.height, b.pitch, 532e-9)
    ctx.upload_cloud(b)
    F = len(frames)
    eager = torch.empty((F, b.height, b.width), device="cuda")
    ctx.batch_compute(frames, eager, mode)           # null stream: never captured
    torch.cuda.synchronize()
    ref = eager.cpu()
    side = torch.cuda.Stream()
    out = torch.empty_like(eager)
    one = torch.empty((b.height, b.width), device="cuda")
    two = torch.empty((2, b.height, b.width), device="cuda")
    codes = torch.empty((b.height, b.width), dtype=torch.uint8, device="cuda")
    for rep in range(4):
        say(f"replay {rep}")
        out.fill_(-1.0)
        torch.cuda.synchronize()
        ctx.batch_compute(frames, out, mode, stream=side)
        side.synchronize()
        assert torch.equal(out.cpu(), ref), f"replay {rep}"
        # single-hologram calls on the same context, on the default stream
        ctx.compute(one, mode)
        ctx.compute_complex(two, mode)
        ctx.kinoform(codes, mode)
        if rep == 1:
            ctx.tune(mode, repeats=1)
        torch.cuda.synchronize()
    ctx.close()
