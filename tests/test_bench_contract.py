"""CPU tests of bench.py's contract and of the counter records it reports:
one GPU only, the rocprofv3 summaries' arithmetic, and committed records
that belong to the current step-kernel sources."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def _pmc_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (kernel, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter,
                        "Counter_Value": value})


def test_counter_traffic_scaled_by_the_copy_probe(tmp_path, monkeypatch):
    """FETCH_SIZE and WRITE_SIZE per step dispatch, each scaled by what the
    same counter reads for the 768 MiB probe copy, in bytes per launch."""
    step = "void ilg::step_kernel<3, unsigned short, 2, 8, 1024, true, false, 10, false>(x)"
    copy = "__amd_rocclr_copyBuffer"
    probe_kib = 768 * 1024
    _pmc_csv(tmp_path / "f.csv", "FETCH_SIZE",
             [(step, 100.0), (step, 102.0), (copy, probe_kib / 2), (copy, 10.0)])
    _pmc_csv(tmp_path / "w.csv", "WRITE_SIZE", [(step, 300.0), (copy, probe_kib)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_file", lambda length: str(out))
    bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1 << 10)
    rec = json.load(open(out))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_bytes_per_launch"] == 101.0 * 2 * 1024
    assert rec["write_bytes_per_launch"] == 300.0 * 1024
    assert rec["bytes_per_launch"] == (202.0 + 300.0) * 1024
    assert rec["alg_bytes_per_launch"] == 12 << 10
    assert rec["step_source_sha256_16"] == bench.step_source_digest()


def test_sq_record_skips_the_first_dispatches(tmp_path, monkeypatch):
    step = "void ilg::step_kernel<3, unsigned short, 2, 8, 1024, true, false, 10, false>(x)"
    path = tmp_path / "sq.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i in range(6):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": step, "Counter_Name": "SQ_INSTS_VALU",
                        "Counter_Value": 1000.0 if i < 2 else 10.0 * i})
            w.writerow({"Dispatch_Id": i, "Kernel_Name": "other", "Counter_Name": "SQ_INSTS_VALU",
                        "Counter_Value": 1e9})
    out = tmp_path / "sq.json"
    monkeypatch.setattr(bench, "SQ_FILE", str(out))
    bench.summarize_sq(str(path), 1 << 10, 2)
    rec = json.load(open(out))
    assert rec["dispatches"] == 4
    assert rec["valu_wave_insts_per_launch"] == (20 + 30 + 40 + 50) / 4


def test_committed_counter_records_match_the_kernel_sources():
    """The traffic and SQ records under profiles/ were taken on the current
    step kernel and sampler sources (bench.py reports `traffic` and
    `alu_roofline` only from such records): a source change needs the
    records retaken with paper_2203_01380_amd/profile_step.sh."""
    for length in (1 << 24, 1 << 26):
        assert bench.counter_traffic(length) is not None, length
        rec = json.load(open(bench.traffic_file(length)))
        assert 1.0 <= rec["bytes_per_launch"] / rec["alg_bytes_per_launch"] < 1.2
    alu = bench.alu_roofline(0.098, 1 << 24)
    assert alu is not None and 0.5 < alu["frac"] < 1.0
    assert 100 < alu["valu_lane_insts_per_node_update"] < 300
