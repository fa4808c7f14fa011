"""Host-side logic of bench.py (no GPU): the byte table of the scheduler
roofline, the stored oracle results of the serving trace, the profile
readers and the one-GPU guard."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_sched_bytes_prices_the_survey_table():
    st = {"tasks": 10, "pushed": 3, "push_batches": 1, "pop_batches": 2, "steal_batches": 1, "data_bytes": 100}
    assert bench.sched_bytes(st) == 76 * 10 + 8 * 3 + 4 * 4 + 100
    st.pop("data_bytes")
    assert bench.sched_bytes(st) == 76 * 10 + 8 * 3 + 4 * 4


def test_sched_roofline_fields():
    tot = {"tasks": 2_000_000, "pushed": 0, "push_batches": 0, "pop_batches": 0, "steal_batches": 0,
           "atomics": 1_000_000}
    r = bench.sched_roofline(tot, 2, [1.0, 1.0], {"distinct": 2e9, "one_word": 1e8}, "")
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 76 * 1_000_000 / 1e-3 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    assert abs(r["atomics"]["achieved_rmw_per_s"] - 5e8) < 1e-3 and abs(r["atomics"]["frac_of_distinct"] - 0.25) < 1e-12


def test_serving_golden_covers_the_whole_trace():
    from synth import serving
    gold = bench.load_serving_golden(20000, 5)
    assert gold is not None and len(gold) == 20000
    specs = serving.serving_mix(20000, 5)
    with open(os.path.join(ROOT, "tests", "golden", "serving_trace_s5.txt")) as fh:
        rows = [ln.split() for ln in fh if not ln.startswith("#")]
    assert [int(r[3]) for r in rows] == gold
    assert [r[1] for r in rows] == [sp.kind for sp in specs]
    assert bench.load_serving_golden(19999, 5) is None and bench.load_serving_golden(20000, 6) is None


def test_profile_readers_check_the_kernel_sources(tmp_path, monkeypatch):
    sha = bench.kernel_source_sha()
    assert sha != bench.kernel_source_sha(bench.BLOCK_KERNEL_SOURCES)
    f = tmp_path / "traffic.txt"
    f.write_text(f"# comment: ignored\nsource_sha: {sha}\nmicrobench.hbm_bytes_per_launch: 123\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("microbench") == 123.0
    assert bench.measured_traffic("serving") is None
    f.write_text("source_sha: 0000\nmicrobench.hbm_bytes_per_launch: 123\n")
    assert bench.measured_traffic("microbench") is None
    v = tmp_path / "valu.txt"
    v.write_text(f"source_sha: {sha}\ntree_daq4.lane_utilisation_pct: 45.5\n")
    monkeypatch.setattr(bench, "VALU_FILE", str(v))
    assert bench.measured_valu() == {"tree_daq4.lane_utilisation_pct": 45.5}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
