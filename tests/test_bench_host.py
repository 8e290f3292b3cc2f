"""bench.py's host-side pieces (no GPU): the one-GPU guard, the counter
summary and its calibration, and the traffic record's source check."""
import json
import os
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _write_pass(folder, counter, rows):
    os.makedirs(folder)
    with open(os.path.join(folder, "run_counter_collection.csv"), "w") as fh:
        fh.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for name, value in rows:
            fh.write('"%s",%s,%r\n' % (name, counter, value))


def test_counter_summary_calibrates_and_sums_the_step(tmp_path, capsys):
    """A 512 MiB copy reading 262144 KiB of FETCH_SIZE gives the factor 2;
    the step's bytes are the per-dispatch mean over its dispatches, scaled."""
    step = "void rc::k_step<0, rc::CellTab>(rc::CellTab, rc::StepParams, rc::StateArgs, rc::OutArgs, long)"
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    _write_pass(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), ("__amd_rocclr_copyBuffer", 1.0),
                                  (step, 1000.0), (step, 3000.0)])
    _write_pass(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 524288.0), (step, 500.0), (step, 500.0)])
    bench.counters_summary(f, w)
    out = capsys.readouterr().out
    rec = json.loads(out.split("traffic-record: ")[1].strip())
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_step"] == pytest.approx(2.0 * 2000.0 * 1024)
    assert rec["write_bytes_per_step"] == pytest.approx(500.0 * 1024)
    assert rec["source_hash"] == bench.source_hash()


def test_traffic_record_is_ignored_for_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "source_hash", lambda: "not-these-sources")
    assert bench.measured_traffic() is None
    assert bench.measured_valu() is None
