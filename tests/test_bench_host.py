"""Host-side logic of bench.py (no GPU): the algorithmic byte accounting of
the force launch and the whole step, the drift estimator, the counter-traffic
guard, the counter summary per form and the one-GPU guard."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_force_bytes_per_particle():
    # count 4, entries 4 n, home position + species 28, v read+write 48,
    # x_ref 24, drifted position 24 (mixed: + the 16-byte record read and written)
    n = 92.0
    assert bench.force_bytes_per_particle(n, False) == pytest.approx(4 + 4 * n + 28 + 48 + 24 + 24)
    assert bench.force_bytes_per_particle(n, False) == pytest.approx(128 + 4 * n)
    assert bench.force_bytes_per_particle(n, True) == pytest.approx(
        4 + 4 * n + (16 + 28) + 48 + 24 + (24 + 16))


def test_step_bytes_add_the_rebuild_share():
    n = 92.0
    f = bench.force_bytes_per_particle(n, False)
    rebuild = 28 + 24 + 160 + 4 * n + 4
    assert bench.step_bytes_per_particle(n, False, 0.0) == pytest.approx(f)
    assert bench.step_bytes_per_particle(n, False, 0.25) == pytest.approx(f + 0.25 * rebuild)


def test_energy_drift_slope_and_short_window():
    # E/N rising by 2e-5 per 1,000 steps plus a constant, logged every step:
    # the slope after the burn-in comes back, with the largest excursion
    n = 1000
    step = 1.0 + np.arange(1100)
    E = n * (3.0 + 2e-8 * step)
    E[:50] += n * 1e-3  # a start-up transient inside the burn-in is ignored
    d = bench.energy_drift(E, n)
    assert d["D"] == pytest.approx(2e-5, rel=1e-6)
    assert d["max_abs_dE_per_particle"] == pytest.approx(2e-8 * 1000, rel=1e-6)
    # fewer than 900 steps after the 100-step burn-in: no figure
    assert bench.energy_drift(E[:900], n) is None


def test_floored_force_error():
    F = np.array([[1.0, 0.0, 0.0], [0.0, 10.0, 0.0]])
    Fo = np.array([[1.0, 0.0, 1e-6], [0.0, 10.0 + 1e-5, 0.0]])
    # particle 0: 1e-6 / max(1, 5); particle 1: 1e-5 / max(10.00001, 5)
    assert bench.floored_force_error(F, Fo, 5.0) == pytest.approx(1e-5 / (10.0 + 1e-5), rel=1e-9)


def test_counter_traffic_needs_the_current_kernel_source(tmp_path, monkeypatch):
    # the counters hold for one force kernel and one list build (the order in
    # which the kernel gathers): a change to either source voids them
    d = {"force_src_sha256": bench.src_sha(), "list_src_sha256": bench.src_sha(bench.LIST_SRC),
         "copy_factor_fetch": 2.0, "copy_factor_write": 1.0,
         "forms": {"fp64": {"fetch_kib": 10.0, "write_kib": 3.0}}}
    p = tmp_path / "c.json"
    p.write_text(json.dumps(d))
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(p))
    assert bench.counters_traffic("fp64") == pytest.approx(10.0 * 1024 * 2.0 + 3.0 * 1024)
    assert bench.counters_traffic("mixed") is None
    for key in ("force_src_sha256", "list_src_sha256"):
        e = dict(d)
        e[key] = "0" * 64
        p.write_text(json.dumps(e))
        assert bench.counters_traffic("fp64") is None


def _write_counters(d, rows):
    """A rocprofv3 --pmc counter_collection.csv with the given (kernel, counter, value) rows."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as f:
        f.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for k, c, v in rows:
            f.write(f'"{k}",{c},{v}\n')


def test_counters_summary_per_form(tmp_path, monkeypatch):
    # the 1M runs give fp64 and mixed (the in-step mode-2 launches only), the
    # 67M run the large mixed form; each counter is scaled by the copy's
    fp64 = "void mdk::k_force<false, 2, 2, 4, false, true>(int)"
    mixed = "void mdk::k_force<true, 2, 1, 8, false, true>(int)"
    tuner = "void mdk::k_force<false, 0, 2, 4, true, true>(int)"
    copy = "__amd_rocclr_copyBuffer"
    t = str(tmp_path)
    _write_counters(t + "/f", [(fp64, "FETCH_SIZE", 100.0), (fp64, "FETCH_SIZE", 300.0),
                               (mixed, "FETCH_SIZE", 50.0), (tuner, "FETCH_SIZE", 1e9)])
    _write_counters(t + "/w", [(fp64, "WRITE_SIZE", 10.0), (mixed, "WRITE_SIZE", 20.0)])
    _write_counters(t + "/cf", [(copy, "FETCH_SIZE", 524288.0)])
    _write_counters(t + "/cw", [(copy, "WRITE_SIZE", 1048576.0)])
    _write_counters(t + "/lf", [(mixed, "FETCH_SIZE", 7000.0)])
    _write_counters(t + "/lw", [(mixed, "WRITE_SIZE", 900.0)])
    out = tmp_path / "c.json"
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(out))
    args = type("A", (), dict(fetch_dir=t + "/f", write_dir=t + "/w", copy_fetch_dir=t + "/cf",
                              copy_write_dir=t + "/cw", large_fetch_dir=t + "/lf",
                              large_write_dir=t + "/lw", commands="test"))()
    bench.counters_summary(args)
    d = json.loads(out.read_text())
    assert d["copy_factor_fetch"] == pytest.approx(2.0)
    assert d["copy_factor_write"] == pytest.approx(1.0)
    assert d["forms"]["fp64"] == {"fetch_kib": 200.0, "write_kib": 10.0, "dispatches": 2}
    assert d["forms"]["mixed"]["fetch_kib"] == 50.0
    assert d["forms"]["large_mixed"] == {"fetch_kib": 7000.0, "write_kib": 900.0, "dispatches": 1}
    assert bench.counters_traffic("large_mixed") == pytest.approx((7000.0 * 2.0 + 900.0) * 1024)
    # without the 67M runs the large form has no counters
    args.large_fetch_dir = None
    bench.counters_summary(args)
    assert "large_mixed" not in json.loads(out.read_text())["forms"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_fp64_flops_need_the_current_kernel_source(tmp_path, monkeypatch):
    src = os.path.join(bench.CSRC, "force_cells.hip")
    d = {"kernels": {"cells_fp64": {"flop_per_dispatch": 2.0e10, "particles": 1000000,
                                    "src_sha256": bench.src_sha(src)}}}
    p = tmp_path / "f.json"
    p.write_text(json.dumps(d))
    monkeypatch.setattr(bench, "FP64_OPS_JSON", str(p))
    assert bench.fp64_flops_per_particle("cells_fp64") == pytest.approx(2.0e4)
    # 2e4 FLOP per particle x 1e6 particles in 1 ms = 20 TFLOP/s
    f = bench.cells_flops(1000000, 1.0)
    assert f["achieved_tflops"] == pytest.approx(20.0)
    assert f["frac"] == pytest.approx(20.0 / 78.6, rel=1e-3)
    d["kernels"]["cells_fp64"]["src_sha256"] = "0" * 64
    p.write_text(json.dumps(d))
    assert bench.fp64_flops_per_particle("cells_fp64") is None
    assert bench.cells_flops(1000000, 1.0) is None
