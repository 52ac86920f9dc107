"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard and the
lookup of measured HBM traffic, which must follow the kernels' sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_traffic_follows_the_sources(tmp_path, monkeypatch):
    # the committed summary, when it matches the current kernel sources, gives more
    # than the algorithmic 404 MB per launch
    t = bench.measured_traffic("spmm_LP", "c2")
    assert t is None or t > 4e8
    assert bench.measured_traffic("spmm_LP", "c3") is None
    # a summary written for other sources is ignored
    text = open(bench.TRAFFIC_FILE).read().replace("    source = ", "    source = 0000")
    stale = tmp_path / "traffic.md"
    stale.write_text(text)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic("spmm_LP", "c2") is None
