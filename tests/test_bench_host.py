"""Host-side logic of bench.py (no GPU): the one-GPU guard, the kernel names
the counter summaries recognise, and the HBM-traffic summary of rocprofv3
counter folders, fed with small synthetic CSV files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("name,key", [
    ("void adr::k_sweep_ws<32, 0, 0, true, true, 384>(adr::SweepParams)", "lsweep"),
    ("void adr::k_sweep_ws<16, 1, 2, false, false, 512>(adr::SweepParams)", "usweep"),
    ("adr::k_pass_xr(adr::IterBufs, adr::BatchGeom)", "pass_xr"),
    ("adr::k_pass_xr_fin(adr::IterBufs, adr::BatchGeom)", None),
    ("void adr::k_pass_v<true>(adr::IterBufs, adr::BatchGeom)", "pass_v"),
    ("adr::k_stream_copy(double __vector(2) const*, double __vector(2)*, long, long)", "copy"),
    ("void (anonymous namespace)::k_conv<32, 0>((anonymous namespace)::ConvArgs)", None),
])
def test_kernel_names(name, key):
    assert bench.kernel_key(name) == key


def _write_pmc(folder, counter, rows):
    """rows: (dispatch id, kernel name, value in KiB)."""
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, v in rows:
            # rocprofv3 reports a counter once per block instance: split the value in two rows
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v / 2})
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v / 2})


def test_traffic_summary_scales_by_the_copy_and_skips_idle_dispatches(tmp_path, monkeypatch, capsys):
    gib_kib = (1 << 30) / 1024.0
    copy = "adr::k_stream_copy(double __vector(2) const*, double __vector(2)*, long, long)"
    lsw = "void adr::k_sweep_ws<32, 0, 0, true, true, 384>(adr::SweepParams)"
    # the copy reads half its bytes by FETCH_SIZE (factor 2) and all of them by WRITE_SIZE (factor 1);
    # the sweep's second dispatch did no work (an instance that had stopped)
    _write_pmc(str(tmp_path / "f"), "FETCH_SIZE", [(1, copy, gib_kib / 2), (2, lsw, 1000.0), (3, lsw, 3.0),
                                                  (4, lsw, 1000.0)])
    _write_pmc(str(tmp_path / "w"), "WRITE_SIZE", [(1, copy, gib_kib), (2, lsw, 500.0), (3, lsw, 1.0),
                                                  (4, lsw, 500.0)])
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "h")
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "traffic", "--pmc-fetch", str(tmp_path / "f"),
                                      "--pmc-write", str(tmp_path / "w"), "--n", "64"])
    args = bench.parse()
    bench.run_traffic(args)
    with open(tmp_path / "profiles" / "traffic.json") as fh:
        t = json.load(fh)
    e = t["n64"]["lsweep"]
    assert e["dispatches"] == 2                      # the idle dispatch is left out
    assert e["fetch_bytes"] == round(1000.0 * 1024 * 2.0)
    assert e["write_bytes"] == round(500.0 * 1024 * 1.0)
    assert e["bytes_per_unknown"] == round((2048000 + 512000) / (64 * 64), 2)
    assert e["source_hash"] == "h"
    assert t["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert "lsweep" in capsys.readouterr().out


def test_forward_pass_counters_are_summed_per_forward(tmp_path):
    h = "void (anonymous namespace)::k_conv<32, 0>((anonymous namespace)::ConvArgs)"
    o = "void (anonymous namespace)::k_conv<16, 1>((anonymous namespace)::ConvArgs)"
    z = "void (anonymous namespace)::k_conv<32, 3>((anonymous namespace)::ConvArgs)"
    rows, d = [], 0
    for rep in range(2):             # two forward passes of 1+...+5 and 10
        for l in range(5):
            d += 1
            rows.append((d, h, float(l + 1)))
        d += 1
        rows.append((d, o, 10.0))
    for l in range(5):               # a training step's forward: other kernels, not counted
        d += 1
        rows.append((d, z, 100.0))
    d += 1
    rows.append((d, o, 100.0))
    _write_pmc(str(tmp_path / "n"), "FETCH_SIZE", rows)
    assert bench.read_forward_pmc(str(tmp_path / "n"), "FETCH_SIZE") == [25.0, 25.0]


def test_source_hash_ignores_comments_and_layout(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text('int f(int x) {  // the lane\'s value\n  return x + 1; /* one\n more */ }\nconst char *s = "a // b";\n')
    b.write_text('// header\nint f(int x) {\n  return x + 1;\n}\nconst char *s = "a // b";   /* kept string */\n')
    c.write_text('int f(int x) { return x + 2; }\nconst char *s = "a // b";\n')
    assert bench.code_text(str(a)) == bench.code_text(str(b))
    assert bench.code_text(str(a)) != bench.code_text(str(c))
    assert '"a // b"' in bench.code_text(str(a))       # a string that looks like a comment stays
