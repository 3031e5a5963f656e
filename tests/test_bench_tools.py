"""bench.py's host-side tools on small synthetic rocprofv3 CSV files (tests/fixtures/rocprof,
made-up numbers): counter scaling by the calibration kernel, the traffic record, and the
per-kernel, per-grid trace summary."""
import json
import os
import shutil

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
FIX = os.path.join(HERE, "fixtures", "rocprof")


def test_ingest_counters_scales_by_calibration(tmp_path, monkeypatch):
    fetch = tmp_path / "fetch"
    write = tmp_path / "write"
    fetch.mkdir()
    write.mkdir()
    shutil.copy(os.path.join(FIX, "fetch_counter_collection.csv"), fetch)
    shutil.copy(os.path.join(FIX, "write_counter_collection.csv"), write)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "feedfacecafebeef")
    table = bench.ingest_counters(str(fetch), str(write))
    # calibration: FETCH reads half of 1 GiB -> factor 2; WRITE exact -> factor 1
    assert "FETCH_SIZE scale 2.0000" in table and "WRITE_SIZE scale 1.0000" in table
    rec = json.load(open(tmp_path / "profiles" / "traffic.json"))
    r = rec["k_sweep2d_tb<double,8,2,3>|blobs2d_4096x4096_f64"]
    assert r["read_bytes"] == int(161000.0 * 1024 * 2)
    assert r["write_bytes"] == int(131072.0 * 1024)
    assert r["bytes_per_launch"] == r["read_bytes"] + r["write_bytes"]
    assert r["kernel_source_sha256_16"] == "feedfacecafebeef"
    # the lookup honours the source hash
    assert bench.measured_traffic("k_sweep2d_tb<double,8,2,3>", "blobs2d_4096x4096_f64") == r["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.measured_traffic("k_sweep2d_tb<double,8,2,3>", "blobs2d_4096x4096_f64") is None


def test_summarize_trace_groups_by_kernel_and_grid():
    table = bench.summarize_trace(FIX)
    lines = [l for l in table.splitlines() if l.startswith("| `")]
    assert len(lines) == 3
    first = [c.strip() for c in lines[0].strip("|").split("|")]
    # two launches of 100 and 96 us on the 194560-thread grid come first (largest total)
    assert first[0] == "`srj::k_sweep2d_tb<double, 8, 2, 3>`" and first[1] == "194560x1x1"
    assert first[2] == "2" and first[4] == "98.00"


def test_kernel_source_hash_skips_comments_only(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1511_04292_amd" / "csrc"
    csrc.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    code = {"sweep2d_tb.hip": "int f(int x)\n{\n    return x + 1;\n}\n", "tb_core.h": "#pragma once\n",
            "formats.h": "struct A { int v; };\n"}

    def write(files):
        for name, text in files.items():
            (csrc / name).write_text(text)
        return bench.kernel_source_hash()

    h0 = write(code)
    commented = dict(code)
    commented["sweep2d_tb.hip"] = ("// header\n/* block\n   comment */\nint f(int x)  // trailing\n{\n\n"
                                   "        return x + 1;\n}\n")
    assert write(commented) == h0
    changed = dict(code)
    changed["sweep2d_tb.hip"] = "int f(int x)\n{\n    return x + 2;\n}\n"
    assert write(changed) != h0
