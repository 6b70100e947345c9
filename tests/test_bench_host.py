"""Host-side checks of bench.py that need no GPU: the one-GPU contract and the
traffic lookup that gates measured bytes on the kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_lookup_is_gated_by_source_hash(tmp_path, monkeypatch):
    rec = {"wl": {"cell_tendency": {"bytes_per_launch": 123,
                                    "source_hash": bench.kernel_source_hash()}},
           "old": {"cell_tendency": {"bytes_per_launch": 456, "source_hash": "0" * 16}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic("cell_tendency", "wl") == 123
    assert bench.measured_traffic("cell_tendency", "old") is None
    assert bench.measured_traffic("vertex_pv", "wl") is None
    assert bench.measured_traffic("cell_tendency", "missing") is None



def test_result_line_is_strict_json():
    """A blown-up run's error (inf or nan) prints as null, not as the
    non-standard Infinity/NaN tokens."""
    out = {"a": float("inf"), "b": [1.5, float("nan"), {"c": -float("inf")}], "d": 2, "e": "x"}
    s = json.dumps(bench.strict(out), allow_nan=False)
    assert json.loads(s) == {"a": None, "b": [1.5, None, {"c": None}], "d": 2, "e": "x"}
