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


def test_max_dt_search_finds_known_limits(capsys):
    """The maximum-time-step procedure on fake contexts whose stability
    limits are known: the largest stable steps come out within the 0.5 %
    bisection tolerance (never above the limit), M is the largest whole
    ratio the coarse limit allows, every run covers the same simulated time,
    and the result line is strict JSON."""
    import types
    import numpy as np
    lim = {"fine": 6.5, "coarse": 40.0, "rk4": 7.9, "rk3": 6.4}
    T = 3600.0

    class Err(Exception):
        pass

    class D:
        def __init__(self, lo, hi):
            self.h_min, self.h_max = lo, hi

    class Ctx:
        def __init__(self):
            self.ok, self.sim = True, 0.0

        def init_state(self, h, u):
            self.ok, self.sim = True, 0.0

        def step(self, dt, M, n):
            self.sim += dt * n
            self.ok &= dt / M <= lim["fine"] and dt <= lim["coarse"]

        def step_scheme(self, s, dt, M, n):
            self.sim += dt * n
            self.ok &= dt <= lim["rk4"]

        def step_rk3(self, dt, n):
            self.sim += dt * n
            self.ok &= dt <= lim["rk3"]

        def diagnostics(self):
            return D(495.0, 505.0)

        def diagnostics_status(self):
            return (0, D(495.0, 505.0)) if self.ok else (-4, D(0.0, 1e9))

        def get_state(self):
            assert abs(self.sim - T) < 1e-6 * T
            return np.full(4, 500.5), None

        def region_counts(self):
            return np.array([100, 10, 10, 50]), None, np.array([5])

        def close(self):
            pass

    mesh = types.SimpleNamespace(nCells=170, areaCell=np.array([1.0, 2.0, 4.0, 3.0]))
    w = types.SimpleNamespace(mesh=mesh, name="fake", M=8, dt_coarse=8 * 2.62,
                              h0=np.full(4, 500.0), u0=None, n_if1=2, n_if2=2)
    saved = bench.timed
    bench.timed = lambda torch, stream, fn: (fn(), 10.0)[1]
    try:
        bench.bench_max_dt(types.SimpleNamespace(max_dt_hours=1.0), w, lambda p: Ctx(),
                           types.SimpleNamespace(LTSError=Err), None, None, "fp64", w.h0, None)
    finally:
        bench.timed = saved
    line = capsys.readouterr().out.strip().splitlines()[-1]
    out = json.loads(line)
    md = out["max_dt"]
    for key, want in (("fine_s", lim["fine"]), ("rk4_s", lim["rk4"]), ("ssprk3_s", lim["rk3"])):
        assert want / 1.006 <= md[key] <= want, (key, md[key])
    assert md["M"] == 6 and md["coarse_s"] <= lim["coarse"]
    assert out["runs"]["lts3_fp64"]["M"] == 6
    assert out["value"] == 0.0 and out["paper_metrics"]["C_cf"] == round(120 / 50, 3)


def test_horizon_steps_cover_the_fixed_time():
    """Every time-to-solution run covers exactly the simulated time, whatever
    its step factor (and whatever --steps), with no step above the asked one."""
    for T in (3600.0, 1234.5):
        for step in (21.4, 5.35, 5.35 / 4, 3600.0, 7.0):
            n, s = bench.horizon_steps(T, step)
            assert abs(n * s - T) <= 1e-9 * T and s <= step * (1 + 1e-12)
            assert n == 1 or (n - 1) * step < T


def test_oracle_baseline_sample_and_parity_state(hex16):
    """The CPU-baseline helper times whole coarse steps of the oracle and hands
    back the state after the first ones, equal to the plain oracle's."""
    import numpy as np
    from oracle import Oracle
    from paper_2106_07154_amd.inputs.workloads import Workload
    from paper_2106_07154_amd.inputs import igw_parameters, igw_state, strip_fine_mask
    m = hex16
    h0, u0 = igw_state(m, igw_parameters(m), 0.0)
    w = Workload("hex16", m, strip_fine_mask(m, 6, 9, 1.0e4), h0, u0, 30.0, 4)
    v, n, t, early, th = bench.oracle_baseline(w, m.nCells * 4, 2, 0.2, first_steps=2)
    assert n >= 2 and v > 0 and th == 2
    o = Oracle(m)
    rh, ru = o.lts(h0, u0, 30.0, 4, o.regions(w.fine_mask, 2, 2), n=2)
    assert np.array_equal(early[0], rh) and np.array_equal(early[1], ru)
