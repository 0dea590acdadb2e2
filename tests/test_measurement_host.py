"""Host logic of the measurement (CPU): the rocprofv3 summaries' copy calibration and per-kernel
averages, the VALU issue time, the algorithmic byte model the roofline divides by, and the
kernel-source hash that keeps counters of other sources out of the bench line."""

import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1305_1505_amd import profile_summary as P  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
X = "void pin::k_xpass<float, 512, 0>(args)"
Y = "void pin::k_ypass_packed<float, 512, 0>(args)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, FIELDS)
        w.writeheader()
        for i, (name, grid, counter, value, t0, t1) in enumerate(rows):
            w.writerow({f: 0 for f in FIELDS} | {"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": grid,
                                                 "Counter_Name": counter, "Counter_Value": value,
                                                 "Start_Timestamp": t0, "End_Timestamp": t1})


def test_traffic_is_scaled_by_the_copy_probe(tmp_path):
    gib = 1 << 30
    # the probe's three 1 GiB copies read as half their bytes (fetch) and all of them (write);
    # a small runtime copy with a smaller grid is not part of the probe
    fetch = [(COPY, 1 << 26, "FETCH_SIZE", gib / 2 / 1024, 0, 1)] * 3 + [(COPY, 64, "FETCH_SIZE", 4.0, 0, 1)]
    fetch += [(X, 1 << 20, "FETCH_SIZE", 1000.0, 0, 1), (X, 1 << 20, "FETCH_SIZE", 3000.0, 0, 1),
              (Y, 1 << 20, "FETCH_SIZE", 500.0, 0, 1)]
    write = [(COPY, 1 << 26, "WRITE_SIZE", gib / 1024, 0, 1)] * 3
    write += [(X, 1 << 20, "WRITE_SIZE", 100.0, 0, 1), (X, 1 << 20, "WRITE_SIZE", 300.0, 0, 1),
              (Y, 1 << 20, "WRITE_SIZE", 50.0, 0, 1)]
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    t = P.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert t["copy_scale_fetch"] == pytest.approx(2.0) and t["copy_scale_write"] == pytest.approx(1.0)
    assert t["kernels"]["xpass_hessian"]["fetch_bytes"] == pytest.approx(2.0 * 1024 * 2000.0)
    assert t["kernels"]["xpass_hessian"]["write_bytes"] == pytest.approx(1024 * 200.0)
    assert t["kernels"]["xpass_hessian"]["dispatches"] == 2
    assert "zpass_collapse" not in t["kernels"]
    assert t["kernel_source_sha256"] == P.kernel_source_hash()


def test_traffic_without_the_probe_is_refused(tmp_path):
    _write(tmp_path / "f.csv", [(X, 1, "FETCH_SIZE", 1.0, 0, 1)])
    _write(tmp_path / "w.csv", [(X, 1, "WRITE_SIZE", 1.0, 0, 1)])
    with pytest.raises(SystemExit, match="copy probe"):
        P.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))


def test_issue_time_is_four_cycles_per_wave_instruction(tmp_path):
    rows = []
    for c, v in (("SQ_WAVES", 1000.0), ("SQ_INSTS_VALU", 2.4e9), ("SQ_INSTS_SALU", 1.0), ("SQ_INSTS_LDS", 1.0),
                 ("SQ_INSTS_VMEM_RD", 1.0), ("SQ_INSTS_VMEM_WR", 1.0)):
        rows.append((Y, 1 << 20, c, v, 0, 2_000_000))
    with open(tmp_path / "sq.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, FIELDS)
        w.writeheader()
        for name, grid, counter, value, t0, t1 in rows:   # one dispatch, one row per counter
            w.writerow({f: 0 for f in FIELDS} | {"Dispatch_Id": 7, "Kernel_Name": name, "Grid_Size": grid,
                                                 "Counter_Name": counter, "Counter_Value": value,
                                                 "Start_Timestamp": t0, "End_Timestamp": t1})
    t = P.issue(str(tmp_path / "sq.csv"))
    k = t["kernels"]["ypass_hessian"]
    # 2.4e9 wave instructions x 4 cycles over 1024 SIMDs at 2.4 GHz
    assert k["valu_issue_ns"] == pytest.approx(2.4e9 * 4 / 1024 / 2.4e9 * 1e9)
    assert k["dispatch_ns"] == 2_000_000 and k["dispatches"] == 1
    assert "| ypass_hessian | 1 | 1000 |" in P.issue_table(t)


def test_algorithmic_bytes_at_512():
    c = 512 * 512 * 256 * 8           # one half slot of complex64
    assert bench.algorithmic_bytes("xpass_hessian", 512, 4) == 4 * c
    assert bench.algorithmic_bytes("ypass_hessian", 512, 4) == 9 * c
    assert bench.algorithmic_bytes("zpass_collapse", 512, 4) == 6 * c + 512 ** 3 * 9
    per_update = (4 * c + 9 * c + 6 * c + 512 ** 3 * 9) / 512 ** 3
    assert per_update == pytest.approx(85.0)
    assert bench.algorithmic_bytes("zpass_collapse", 512, 8) == 6 * 2 * c + 512 ** 3 * 17


def test_committed_counters_are_used_only_for_their_sources(monkeypatch):
    from paper_1305_1505_amd import binding as B

    with open(os.path.join(ROOT, "profiles", "traffic_c512_fp32.json")) as fh:
        committed = json.load(fh)["kernel_source_sha256"]
    monkeypatch.setattr(P, "kernel_source_hash", lambda: committed)
    assert bench.measured_traffic("ypass_hessian", 512, B.PIN_FP32)["bytes"] > 0
    assert bench.measured_issue("zpass_collapse", 512, B.PIN_FP32) > 0
    assert bench.measured_traffic("ypass_hessian", 256, B.PIN_FP32) is None
    assert bench.measured_traffic("ypass_hessian", 512, B.PIN_FP64) is None
    monkeypatch.setattr(P, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic("ypass_hessian", 512, B.PIN_FP32) is None
    assert bench.measured_issue("zpass_collapse", 512, B.PIN_FP32) is None

