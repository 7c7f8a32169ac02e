"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message and exit status 2, before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "--gpus must be 1" in p.stderr
    assert p.stdout.strip() == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="2")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True,
                       text=True, timeout=120, env=env)
    assert p.returncode == 2
    assert "--gpus must be 1" in p.stderr


def test_recorded_traffic_holds_only_for_its_source_and_shape():
    """A counter-measured HBM traffic entry is reported only for the launch
    shape it was taken on and while its kernel source is unchanged (a
    changed source reads as no record, never as stale bytes)."""
    import hashlib
    import sys
    sys.path.insert(0, ROOT)
    import bench

    def current(kernel):
        for t in bench.TRAFFIC:
            if t["kernel"] == kernel:
                with open(os.path.join(bench.ROOT, t["src"]), "rb") as f:
                    return hashlib.sha256(f.read()).hexdigest()[:16] == t["sha"]
        return False

    split = "gfx950/1920x1080/mode1/kb10: bm=384 bn=192 waves=4x2 stages=2 splits=8 rows=0 1 us"
    batch = "gfx950/1920x1080/mode2/batch/kb12: bm=384 bn=192 waves=4x2 stages=2 rows=0 1 us"
    # other shapes and sizes never match a record
    assert bench.traffic_bytes("gemm_split_mfma", split.replace("splits=8", "splits=6")) is None
    assert bench.traffic_bytes("gemm_split_mfma_batch", batch.replace("bm=384", "bm=192")) is None
    assert bench.traffic_bytes("fresnel_diffraction", "2048") is None
    assert bench.traffic_bytes("gemm_split_mfma", None) is None
    # recorded shapes: the calibrated bytes while the source is the recorded one
    rec = next(t for t in bench.TRAFFIC
               if t["kernel"] == "gemm_split_mfma" and t["plan"] == "384,192,4,2,2,8")
    want = ((rec["fetch_kib"] * bench.TRAFFIC_SCALE["fetch"] +
             rec["write_kib"] * bench.TRAFFIC_SCALE["write"]) * 1024.0
            if current("gemm_split_mfma") else None)
    assert bench.traffic_bytes("gemm_split_mfma", split) == want
    if want is not None:
        assert 2.5e8 < want < 5e8      # factor reads and split partials, not more
    other = split.replace("bm=384 bn=192 waves=4x2", "bm=192 bn=320 waves=2x4").replace(
        "splits=8", "splits=7")
    got = bench.traffic_bytes("gemm_split_mfma", other)
    assert (got is not None and got != want) if current("gemm_split_mfma") else got is None
    got = bench.traffic_bytes("gemm_split_mfma_batch", batch)
    assert (got is not None and got > 4e10) if current("gemm_split_mfma_batch") else got is None
    got = bench.traffic_bytes("fresnel_diffraction", "1024")
    assert (got is not None and got > 3e7) if current("fresnel_diffraction") else got is None
