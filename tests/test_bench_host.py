"""Host logic of bench.py that needs no GPU: the one-GPU guard, the tuner-line
parser and the counter-record lookup behind the roofline's traffic figure."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("line,key", [
    ("chosen: split layout target_wgs=1024 work_items=1024 slots=16 (30.78 us/eval) key=x", "split/1024"),
    ("chosen: small-member layout target_wgs=0 work_items=256 slots=1 (9.1 us/eval) key=x", "small/256"),
    ("chosen: spatial split layout target_wgs=32768 work_items=32768 slots=8 (49.8 us/eval) key=x",
     "spatial/32768"),
    ("cached choice", None),
    (None, None),
])
def test_layout_key(line, key):
    assert bench.layout_key(line) == key


def test_traffic_record_lookup(tmp_path, monkeypatch):
    digest = bench.force_sources_digest()
    f = tmp_path / "counters.md"
    f.write_text("# summary\n\n```\n"
                 f"traffic kernel=k_forces<float,true> workload=twisted_rod precision=mixed "
                 f"layout=split/1024 sources={digest} bytes_per_launch=1234\n"
                 f"traffic kernel=k_forces<float,true> workload=twisted_rod precision=mixed "
                 f"layout=split/512 sources=0000000000000000 bytes_per_launch=99\n```\n")
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(f))
    assert bench.measured_traffic("k_forces<float, true>", "twisted_rod", "mixed", "split/1024") == 1234
    # other layout, stale sources, other workload or precision: no figure
    assert bench.measured_traffic("k_forces<float, true>", "twisted_rod", "mixed", "split/512") is None
    assert bench.measured_traffic("k_forces<float, true>", "ensemble", "mixed", "split/1024") is None
    assert bench.measured_traffic("k_forces<float, true>", "twisted_rod", "fp64", "split/1024") is None
    assert bench.measured_traffic("k_forces<float, true>", "twisted_rod", "mixed", None) is None


def test_digest_covers_the_force_kernel_sources():
    csrc = os.path.join(ROOT, "paper_2603_27279_amd", "csrc")
    for name in bench.FORCE_SOURCES:
        assert os.path.exists(os.path.join(csrc, name)), name
    assert "k_forces.hip" in bench.FORCE_SOURCES and "dipole_body.h" in bench.FORCE_SOURCES


@pytest.mark.parametrize("gsteps,steps,plan", [
    (200, 20, (20, 20, 0)), (200, 2000, (200, 2000, 0)), (100, 250, (100, 200, 50)),
    (0, 20, (0, 0, 20)), (5, 5, (5, 5, 0))])
def test_graph_plan_replays_whole_graphs(gsteps, steps, plan):
    assert bench.graph_plan(gsteps, steps) == plan


@pytest.mark.parametrize("rows", [False, True])
def test_cpu_baseline_reports_cores_model_and_one_core(monkeypatch, rows):
    import workloads
    if rows:  # sample by rows, as for the largest workloads
        monkeypatch.setattr(bench, "ROW_SAMPLE_PAIRS", 0)
    w = workloads.twisted_rod(n=300)
    cb = bench.cpu_baseline(w, target_s=0.3)
    assert cb["kind"] == "oracle" and cb["unit"] == "particle-steps/s"
    assert cb["value"] > 0 and cb["one_core"]["value"] > 0 and cb["cores"] >= 1
    assert ("dipole and contact sums" in cb["sample"]) == rows
    assert "logical_cpus" in cb and "cpu_model" in cb


def test_member0_slices_the_first_ensemble_member():
    import numpy as np
    import workloads
    w = workloads.ensemble(members=3, n=50)
    v = bench._member0(w)
    assert v["n"] == 50 and v["n_members"] == 1 and list(v["rod_offset"]) == [0, 50]
    assert v["field"].shape == (w["field"].shape[0], 1, 12)
    np.testing.assert_array_equal(v["x0"], w["x0"][:50])
    np.testing.assert_array_equal(v["rod_params"], w["rod_params"][:1])


def test_oracle_timings_rows_and_thread_restore(monkeypatch):
    """--oracle-timings: one row per workload and thread count (the rod array on
    all threads only), rates from the steps timed, and the oracle's thread count
    set back afterwards. Every workload is replaced by the 20-particle
    cantilever so that the test runs in seconds."""
    import ctypes
    import oracle
    import workloads
    monkeypatch.setattr(workloads, "make", lambda name, **kw: workloads.cantilever())
    lib = oracle._load()
    lib.orc_threads.restype = ctypes.c_int
    before = int(lib.orc_threads())
    r = bench.oracle_timings()
    assert int(lib.orc_threads()) == before == r["threads"]
    names = [(x["workload"], x["threads"]) for x in r["rows"]]
    assert names[:5] == [(n, before) for n in ("cantilever", "adjoint_rod", "twisted_rod",
                                               "cilia_carpet", "rod_array")]
    assert ("rod_array", 1) not in names and len(names) == 9
    for x in r["rows"]:
        assert x["seconds"] > 0
        assert x["particle_steps_per_s"] == pytest.approx(20 * x["steps"] / x["seconds"])
        assert x["dipole_pair_evals_per_s"] == pytest.approx(380 * x["steps"] / x["seconds"])
