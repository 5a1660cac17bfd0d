"""bench.py's command-line contract, checked without a GPU: one GPU only
(any other --gpus exits with a message before touching a device), and the
algorithmic byte counts its roofline uses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    n, npart = 512, 512 ** 3
    b = bench.algorithmic_bytes(n, npart, 4)
    grid = 4 * n ** 3 * 4
    assert b["moments+count"] == 24 * npart
    assert b["permute"] == (24 + 24) * npart          # float32 pos + vel in, 24-byte records out
    assert b["clear"] == grid
    assert b["scatter"] == 24 * npart + grid
    assert b["fft_z"] == b["fft_y"] == 2 * grid


def test_scatter_traffic_needs_its_source():
    """The measured scatter traffic is reported only with the hash of the
    kernel source it was measured on, and only while that source is unchanged."""
    sys.path.insert(0, ROOT)
    import bench
    t = dict(bench.SCATTER_TRAFFIC)
    try:
        bench.SCATTER_TRAFFIC["source_sha16"] = "0" * 16
        assert bench.scatter_traffic() is None
        bench.SCATTER_TRAFFIC["source_sha16"] = bench._sha16(t["source"])
        got = bench.scatter_traffic()
        assert got["bytes"] == t["bytes"] and got["profile"] == t["profile"]
    finally:
        bench.SCATTER_TRAFFIC.clear()
        bench.SCATTER_TRAFFIC.update(t)
