"""Host-side checks of bench.py (no GPU): the one-GPU rule and the counter
summary written from two rocprofv3 --pmc CSV files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_counter_ingest(tmp_path, monkeypatch):
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    out = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(out))
    nx, ny, nz = 64, 32, 16
    N = nx * ny * nz
    known_kib = 19 * N * 4 / 1024.0  # the sweep's algorithmic reads (and writes)
    from paper_0811_4593_amd import lbm
    copy_kib = lbm.lbm_buffer_elements(nx, ny, nz, lbm.LBM_STORE_F32, lbm.LBM_LAYOUT_ROW_MAJOR) * 4 / 1024.0  # the whole buffer
    sweep = "void lbm::sweep_kernel<lbm::FormF32, 256, 1, true, false, false>(float const*, float*, args)"
    pull = "void lbm::sweep_kernel<lbm::FormF32, 256, 1, true, true, false>(float const*, float*, args)"
    copy = "lbm::copy_probe_kernel(uint4 const*, uint4*, unsigned long)"
    # counters read half the fetched bytes and all written bytes (the ratios measured on MI355X)
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(sweep, known_kib / 2 * 1.01), (sweep, known_kib / 2 * 0.99),
                                            (pull, 1.0), (copy, copy_kib / 2)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(sweep, known_kib), (pull, 1.0), (copy, copy_kib)])

    class A:
        ingest_counters = (str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
        storage = "f32"
        nx, ny, nz = 64, 32, 16
        launch = "256,1,1"
        layout = "rows"
        counters_command = "test"
        steps_per_pass, zplanes, tile_rows = 1, 0, 0

    bench.ingest_counters(A)
    rec = json.loads(out.read_text())
    assert rec["kernel"] == sweep
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(rec["algorithmic_bytes_per_launch"], rel=1e-12)
    assert rec["launch"] == [256, 1, 1] and rec["kernel_source_hash"] == bench.kernel_source_hash()
    assert rec["layout"] == "rows"
    # the figures are used only for the layout, launch and storage they were taken on
    assert bench.measured_traffic([256, 1, 1], "f32", "rows") == rec["hbm_bytes_per_launch"]
    assert bench.measured_traffic([256, 1, 1], "f32", "pop") is None
    assert bench.measured_traffic([128, 1, 1], "f32", "rows") is None


def test_counter_ingest_two_step_pass(tmp_path, monkeypatch):
    """A run with two steps per pass is summarised on the two-step kernel,
    whose algorithmic bytes per launch are those of two steps."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod2", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    out = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(out))
    from paper_0811_4593_amd import lbm
    nx, ny, nz = 64, 32, 16
    N = nx * ny * nz
    copy_kib = lbm.lbm_buffer_elements(nx, ny, nz, lbm.LBM_STORE_F32, lbm.LBM_LAYOUT_ROW_MAJOR) * 4 / 1024.0
    k2 = "void lbm::sweep2_kernel<lbm::FormF32, 13>(float const*, float*, args)"
    k1 = "void lbm::sweep_kernel<lbm::FormF32, 256, 1, true, false, false>(float const*, float*, args)"
    copy = "lbm::copy_probe_kernel(uint4 const*, uint4*, unsigned long)"
    per_step_kib = 19 * N * 4 / 1024.0
    # one launch of the pass reads 1.1 times and writes once the populations of the nodes
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(k2, 1.1 * per_step_kib / 2), (k1, 1.0), (copy, copy_kib / 2)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(k2, per_step_kib), (k1, 1.0), (copy, copy_kib)])

    class A:
        ingest_counters = (str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
        storage = "f32"
        nx, ny, nz = 64, 32, 16
        launch = "256,1,1"
        layout = "rows"
        counters_command = "test"
        steps_per_pass, zplanes, tile_rows = 2, 32, 0

    bench.ingest_counters(A)
    rec = json.loads(out.read_text())
    assert rec["kernel"] == k2 and rec["steps_per_launch"] == 2
    assert rec["algorithmic_bytes_per_launch"] == 2 * 2 * 19 * N * 4
    assert rec["hbm_bytes_per_launch"] == pytest.approx(2.1 * 19 * N * 4, rel=1e-12)
    assert bench.measured_traffic([256, 1, 1], "f32", "rows", 2, [2, 32, 0]) == rec["hbm_bytes_per_launch"]
    assert bench.measured_traffic([256, 1, 1], "f32", "rows", 1, [1, 0, 0]) is None
    assert bench.measured_traffic([256, 1, 1], "f32", "rows", 2, [2, 64, 0]) is None
