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


FIRST = "void rc::k_newton_first<rc::CellTab>(rc::CellTab, rc::StepParams, rc::StateArgs, rc::OutArgs, rc::ResumeArgs, long)"
SORT = "rc::k_tile_sort(rc::ResumeArgs, long)"
RESUME = "void rc::k_newton_resume<rc::CellTab>(rc::CellTab, rc::StepParams, rc::StateArgs, rc::OutArgs, rc::ResumeArgs)"


def test_counter_summary_calibrates_and_sums_the_step(tmp_path, capsys):
    """A 512 MiB copy reading 262144 KiB of FETCH_SIZE gives the factor 2; a
    step's bytes are the sum over its launches (first pass, tile sort,
    resumed pass) per step, scaled; the SQ pass gives VALU instructions per step."""
    f, w, q = str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "q")
    _write_pass(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), ("__amd_rocclr_copyBuffer", 1.0),
                                  (FIRST, 1000.0), (SORT, 10.0), (RESUME, 2000.0),
                                  (FIRST, 3000.0), (SORT, 30.0), (RESUME, 4000.0),
                                  ("rc::k_step<2, rc::CellTab>(...)", 1e9)])
    _write_pass(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 524288.0), (FIRST, 500.0), (SORT, 1.0),
                                  (RESUME, 100.0), (FIRST, 500.0), (SORT, 1.0), (RESUME, 100.0)])
    os.makedirs(q)
    with open(os.path.join(q, "run_counter_collection.csv"), "w") as fh:
        fh.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for k, valu in ((FIRST, 2000.0), (SORT, 10.0), (RESUME, 1000.0)):
            for c, v in (("SQ_WAVES", 100.0), ("SQ_INSTS_VALU", valu), ("SQ_INSTS_SALU", 1.0),
                         ("SQ_INSTS_VMEM_RD", 1.0), ("SQ_ACTIVE_INST_VALU", 1.0), ("SQ_WAVE_CYCLES", 10.0),
                         ("SQ_WAIT_INST_ANY", 1.0), ("SQ_BUSY_CYCLES", 1.0), ("GRBM_GUI_ACTIVE", 8 * 2.4e6)):
                fh.write('"%s",%s,%r\n' % (k, c, v))
    bench.counters_summary(f, w, q)
    out = capsys.readouterr().out
    rec = json.loads(out.split("traffic-record: ")[1].strip())
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_step"] == pytest.approx(2.0 * (4000.0 + 40.0 + 6000.0) / 2 * 1024)
    assert rec["write_bytes_per_step"] == pytest.approx(601.0 * 1024)
    assert rec["valu_insts_per_step"] == pytest.approx(3010.0)
    assert rec["source_hash"] == bench.source_hash()


def test_trace_summary_skips_warmup(tmp_path, capsys):
    d = tmp_path / "t"
    d.mkdir()
    with open(d / "run_kernel_trace.csv", "w") as fh:
        fh.write("Kernel_Name,Start_Timestamp,End_Timestamp,Workgroup_Size_X\n")
        t = 0
        for dur in (5000, 1000, 1000):
            for k, frac in ((FIRST, 0.5), (SORT, 0.1), (RESUME, 0.4)):
                fh.write('"%s",%d,%d,64\n' % (k, t, t + int(dur * frac)))
                t += 10000
    bench.trace_summary(str(d), 1)
    out = capsys.readouterr().out
    assert "Newton step, two-pass form (sum of the averages of its launches): 1.0 us" in out
    assert "| `void rc::k_newton_first<rc::CellTab>` | 64 | 2 | 1 | 0.5 |" in out


def test_short_name_drops_the_parameter_list():
    assert bench.short_name("rc::(anonymous namespace)::k_nodes4d(rc_axes4, float*)") == "rc::k_nodes4d"
    assert bench.short_name("void rc::k_step<0, rc::CellTab>(rc::CellTab, long)") == "void rc::k_step<0, rc::CellTab>"


def test_traffic_record_is_ignored_for_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "source_hash", lambda: "not-these-sources")
    assert bench.measured_traffic() is None
    assert bench.valu_roofline(1.0) is None
