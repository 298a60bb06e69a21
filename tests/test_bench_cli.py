"""Host-side argument handling of bench.py (no GPU: both cases exit before torch loads)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _run(*args):
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True,
                          timeout=60, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_hardware_queue_count_is_range_checked():
    for bad in ("0", "1", str(32 + 1)):
        r = _run("--hw-queues", bad)
        assert r.returncode == 2
        assert "--hw-queues" in r.stderr


def test_traffic_is_reported_only_for_the_profiled_stream_source(monkeypatch):
    """bench.py reports the counter-measured HBM bytes of the stream pass only while the
    stream pass's source still has the digest the committed summary was taken with; the
    bytes are FETCH_SIZE and WRITE_SIZE scaled by the copy calibration."""
    sys.path.insert(0, ROOT)
    import bench
    t = bench.measured_traffic()
    assert t is not None and 1.0 < t / bench.STREAM_BYTES_PER_ELEM / 8192 ** 2 < 1.2
    monkeypatch.setattr(bench, "stream_source_digest", lambda: "0000000000000000")
    assert bench.measured_traffic() is None
