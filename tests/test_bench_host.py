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


def _golden():
    with open(os.path.join(ROOT, "tests", "golden", "paper_cost_metrics.json")) as f:
        return json.load(f)


def test_paper_optimal_ratio_matches_printed_value():
    """The paper's worked example of its ideal LTS speed-up (fixture cites it):
    474,467 coarse time-step cells, 146,540 fine ones, M = 4 -> 2.342."""
    g = _golden()["optimal_ratio"]
    r = bench.paper_optimal_ratio(g["coarse_step_cells"], g["fine_cells"], g["M"])
    assert round(r, g["decimals"]) == g["value"]
    # M = 1 gains nothing; all cells fine gains nothing
    assert bench.paper_optimal_ratio(1000, 500, 1) == 1.0
    assert bench.paper_optimal_ratio(0, 500, 8) == 1.0


def test_paper_cell_ratio_and_gain_match_printed_values():
    """C_cf of the three region setups and the gain column of the RK4
    comparison table, recomputed from the printed cell counts and CPU times.
    The printed gains are cut to three decimals from the unrounded times, so
    they are held to one unit in the last place."""
    g = _golden()
    for c in g["C_cf"]["cases"]:
        assert abs(bench.coarse_fine_ratio(c["coarse_step_cells"], c["fine_cells"]) - c["value"]) < 1e-3
    for c in g["gain_percent"]["cases"]:
        for t, want in zip(c["lts3"], c["gain"]):
            assert abs(bench.gain_percent(c["rk4"], t) - want) < 1e-3, (c["ranks"], t)


def test_area_ratio():
    import numpy as np
    from paper_2106_07154_amd.inputs import periodic_hex_mesh
    m = periodic_hex_mesh(8, 8, 1.0e4)
    assert abs(bench.area_ratio(m.areaCell) - 1.0) < 1e-12
    assert bench.area_ratio(np.array([2.0, 0.5, 1.0])) == 4.0
