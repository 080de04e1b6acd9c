"""bench.py's host-side contract: one GPU only, and the HBM traffic figure comes
from the committed counter summary only while the aggregation sources are the
ones it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_traffic_figure_follows_the_source_hash(tmp_path, monkeypatch):
    import bench
    v = bench.measured_traffic()
    text = open(bench.TRAFFIC_PROFILE).read()
    if bench.aggregation_source_hash() in text:
        # taken on these sources: at least the path values the pass writes
        assert isinstance(v, int) and v > 944_000_000
    else:
        assert v is None
    # a summary recorded for other sources is not used
    other = tmp_path / "traffic.md"
    other.write_text(text.replace(bench.aggregation_source_hash(), "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(other))
    assert bench.measured_traffic() is None
