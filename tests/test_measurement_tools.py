"""Host logic of the measurement tools: the counter summaries (traffic.py) on
small synthetic rocprofv3 CSVs, and the bench's algorithmic byte counts."""
import csv
import json
import os
import sys
import types

import pytest

from paper_2310_07119_amd import traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KICK = "void tw::pass_kernel<double, 512, 5, true>(tw::PassArgs)"
DECOY = "void tw::pass_kernel<float, 512, 5, true>(tw::PassArgs)"
COPY = "__amd_rocclr_copyBuffer"
FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_summarize_scales_by_the_copy_calibration(tmp_path):
    # two kick dispatches, each counter split over two instances (summed per dispatch),
    # and an FP32 kernel of the same kind that must not be counted
    _csv(tmp_path / "fetch", [(1, KICK, "FETCH_SIZE", 600.0, 0, 1), (1, KICK, "FETCH_SIZE", 400.0, 0, 1),
                              (2, KICK, "FETCH_SIZE", 1200.0, 0, 1), (3, DECOY, "FETCH_SIZE", 9e9, 0, 1)])
    _csv(tmp_path / "write", [(1, KICK, "WRITE_SIZE", 700.0, 0, 1), (2, KICK, "WRITE_SIZE", 900.0, 0, 1)])
    mib = 64
    # the copy moves 64 MiB each way; the fetch counter reads half of it, the write counter all of it
    _csv(tmp_path / "cf", [(1, COPY, "FETCH_SIZE", mib * 1024 / 2, 0, 1)])
    _csv(tmp_path / "cw", [(1, COPY, "WRITE_SIZE", mib * 1024, 0, 1)])
    out = tmp_path / "t.json"
    a = types.SimpleNamespace(fetch=str(tmp_path / "fetch"), write=str(tmp_path / "write"),
                              copy_fetch=str(tmp_path / "cf"), copy_write=str(tmp_path / "cw"), out=str(out),
                              kind="pass_kick_drift", precision="fp64", length=512, copy_mib=mib, commands="c")
    traffic.summarize(a)
    d = json.load(open(out))
    assert d["dispatches"] == [2, 2]
    assert d["copy_scale"]["fetch"] == pytest.approx(2.0) and d["copy_scale"]["write"] == pytest.approx(1.0)
    assert d["fetch_bytes_per_launch"] == pytest.approx(1100.0 * 1024 * 2)
    assert d["write_bytes_per_launch"] == pytest.approx(800.0 * 1024)
    assert d["source_digest"] == traffic.source_digest()
    assert os.path.exists(tmp_path / "t.md")


def test_counters_derived_figures(tmp_path):
    # one dispatch of 1 ms: GRBM summed over 8 XCDs, 256 CUs
    g = 8 * 1000.0
    rows = [(1, KICK, "GRBM_GUI_ACTIVE", g, 0, 1_000_000), (1, KICK, "SQ_ACTIVE_INST_VALU", 256 * 1000.0 * 0.4, 0, 1_000_000),
            (1, KICK, "SQ_LDS_IDX_ACTIVE", 256 * 1000.0 * 0.3, 0, 1_000_000),
            (1, KICK, "SQ_LDS_BANK_CONFLICT", 256 * 1000.0 * 0.1, 0, 1_000_000),
            (1, KICK, "SQ_INSTS_VALU_ADD_F64", 1e6, 0, 1_000_000), (1, KICK, "SQ_INSTS_VALU_MUL_F64", 1e6, 0, 1_000_000),
            (1, KICK, "SQ_INSTS_VALU_FMA_F64", 1e6, 0, 1_000_000)]
    _csv(tmp_path / "p", rows)
    out = tmp_path / "c.md"
    a = types.SimpleNamespace(dirs=[str(tmp_path / "p")], out=str(out), precision="fp64", length=512, title="t",
                              commands="c", cus=256, xcds=8, raw=["SQ_INSTS_VALU"])
    traffic.counters(a)
    text = open(out).read()
    line = [l for l in text.splitlines() if l.startswith("| `void tw::pass_kernel<double, 512, 5")][0]
    cells = [c.strip() for c in line.split("|")]
    # VALU busy 40%; FLOP/s = 64 * (1 + 1 + 2) * 1e6 / 1 ms = 0.256 TFLOP/s; LDS 30%, conflicts 10%, 0.5 per access
    assert cells[4] == "40.0%" and cells[5] == "0.26" and cells[6] == "30.0%" and cells[7] == "10.0%"
    assert cells[8] == "0.50"


def test_counters_from_several_runs_are_not_added(tmp_path):
    # GRBM_GUI_ACTIVE in each of two counter runs with the same dispatch ids:
    # each run's value is one dispatch's, so the VALU share stays 40%
    g = 8 * 1000.0
    _csv(tmp_path / "a", [(1, KICK, "GRBM_GUI_ACTIVE", g, 0, 1_000_000),
                          (1, KICK, "SQ_ACTIVE_INST_VALU", 256 * 1000.0 * 0.4, 0, 1_000_000)])
    _csv(tmp_path / "b", [(1, KICK, "GRBM_GUI_ACTIVE", g, 0, 1_000_000),
                          (1, KICK, "SQ_WAIT_ANY", 250.0, 0, 1_000_000), (1, KICK, "SQ_WAVE_CYCLES", 1000.0, 0, 1_000_000),
                          (1, KICK, "SQ_ACTIVE_INST_ANY", 300.0, 0, 1_000_000)])
    out = tmp_path / "c.md"
    a = types.SimpleNamespace(dirs=[str(tmp_path / "a"), str(tmp_path / "b")], out=str(out), precision="fp64",
                              length=512, title="t", commands="c", cus=256, xcds=8, raw=["GRBM_GUI_ACTIVE"])
    traffic.counters(a)
    line = [l for l in open(out).read().splitlines() if l.startswith("| `void tw::pass_kernel<double, 512, 5")][0]
    cells = [c.strip() for c in line.split("|")]
    assert cells[4] == "40.0%"
    assert cells[9] == "25.0%" and cells[10] == "30.0%"   # waiting and issuing shares of the wave time


def test_kernel_summary_selects_the_timed_launches(tmp_path):
    # a trace with 3 warmup, 2 timed and 2 re-profiled launches of the kick pass:
    # --timed-launches 2 --skip-last 2 averages the timed ones
    d = tmp_path / "kt"
    os.makedirs(d)
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"])
        w.writeheader()
        w.writerow(dict(Name=KICK, Calls=7, TotalDurationNs=1, AverageNs=1, Percentage=100, MinNs=1, MaxNs=1))
    durs = [900, 900, 900, 500, 700, 100, 100]
    with open(d / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for u in durs:
            w.writerow(dict(Kernel_Name=KICK, Start_Timestamp=t, End_Timestamp=t + u * 1000))
            t += 10_000_000
    out = tmp_path / "k.md"
    a = types.SimpleNamespace(dir=str(d), out=str(out), command="c", title="t", bench_log="", timed_launches=2,
                              skip_last=2, top=5)
    traffic.kernels(a)
    rows = [l for l in open(out).read().splitlines() if l.startswith("| fp64 | pass_kick_drift | 2 |")]
    assert rows and "600.0" in rows[0]


def test_bench_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    ncell, nfield = 512 * 512, 257
    npairs = (nfield + 1) // 2
    f, z = 16 * ncell * nfield, 16 * ncell * npairs
    assert bench.pass_bytes("pass_kick_drift", 16, ncell, nfield, 256) == z + 2 * f == 2696937472
    assert bench.pass_bytes("pass_drift_rho", 16, ncell, nfield, 256) == 2 * f + z
    assert bench.pass_bytes("pass_zpoisson", 16, ncell, nfield, 256) == 2 * z
    assert bench.pass_bytes("no_such_kind", 16, ncell, nfield, 256) is None


def test_bench_traffic_needs_matching_kernel_sources(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    fn = os.path.join(ROOT, "profiles", "traffic_pass_kick_drift_2d_n512_pair_fp64.json")
    stored = json.load(open(fn))
    monkeypatch.setattr(traffic, "source_digest", lambda: stored["source_digest"])
    assert bench.measured_traffic("pass_kick_drift", "fp64", "2d_n512_pair") == stored["traffic_bytes_per_launch"]
    monkeypatch.setattr(traffic, "source_digest", lambda: "changed")
    assert bench.measured_traffic("pass_kick_drift", "fp64", "2d_n512_pair") is None
    assert bench.measured_traffic("pass_kick_drift", "fp64", "no_such_workload") is None


def test_bench_roofline_uses_algorithmic_bytes_per_cell_step():
    """The roofline's achieved rate is 32 B (FP64) per realization*cell*step
    times the cells one launch covers, over the dominant kernel's average
    launch; the step figures add up every step pass from a steps-only profile."""
    import bench
    ncell, nfield, n_real = 512 * 512, 257, 256
    prof = {"pass_kick_drift": (50, 50 * 0.5), "pass_drift_rho": (51, 51 * 0.45), "pass_zpoisson": (51, 51 * 0.25),
            "sample": (1, 0.9)}
    step_prof = {"steps": 50, "prof": {"pass_kick_drift": (50, 25.0), "pass_drift_rho": (50, 22.5),
                                       "pass_zpoisson": (50, 12.5), "pass_drift": (1, 0.4)}}
    r = bench.roofline_of(prof, "fp64", 16, ncell, nfield, n_real, 50, step_prof, ms_per_step=1.5)
    alg = 32 * nfield * ncell
    assert r["kernel"] == "pass_kick_drift" and r["alg_bytes_per_launch"] == alg
    assert abs(r["achieved"] - alg / 0.5e-3 / 1e9) < 1e-9 * r["achieved"]
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-15
    assert abs(r["step_frac"] - alg / 1.5e-3 / 1e9 / 8000.0) < 1e-12
    assert abs(r["step_kernel_ms"] - (25.0 + 22.5 + 12.5 + 0.4) / 50) < 1e-12
    # 2D FP64 schedule: drift+rho 2f + z, Poisson 2z, kick 2f + z per step (f: every field once, z: the
    # pair scratch once, 129 pairs for 257 fields: about 96 B per field*cell), plus one opening drift
    f, z = 16 * ncell * nfield, 16 * ncell * 129
    per_cs = (50 * (4 * f + 4 * z) + 2 * f) / (50 * nfield * ncell)
    assert 96.6 < per_cs < 96.8
    assert abs(r["pass_bytes_per_cell_step"] - per_cs) < 1e-9
    assert abs(r["pass_bytes_ratio"] - per_cs / 32) < 1e-9
    assert bench.alg_bytes_per_cell_step("fp32") == 16
