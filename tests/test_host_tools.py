"""Host-side logic of the measurement tools (CPU only): the rocprofv3 summaries
kept with the profiles, the traffic record bench.py reads, and bench.py's
algorithmic-byte count, bridge share and multi-threaded oracle timing."""
import csv
import os
import shutil
import sys
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_1312_3062_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_traffic_scales_each_counter_by_the_copy_kernel(tmp_path):
    gib = 1 << 30
    # the copy kernel moves 1 GiB each way; FETCH_SIZE reads half of it, WRITE_SIZE all (KiB)
    copy = "void at::native::bitwise_not_kernel(int*)"
    search = "void ann::(anonymous namespace)::k_search<0, 8, 1, false, false>(ann::SearchArgs)"
    fetch = [(1, copy, "FETCH_SIZE", gib / 1024 / 2), (2, search, "FETCH_SIZE", 1000.0),
             (3, search, "FETCH_SIZE", 3000.0)]
    write = [(1, copy, "WRITE_SIZE", gib / 1024), (2, search, "WRITE_SIZE", 10.0), (3, search, "WRITE_SIZE", 30.0)]
    _write_counters(tmp_path / "f.csv", fetch)
    _write_counters(tmp_path / "w.csv", write)
    r = profiling.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), r"k_search<0, 8, 1, false, false>",
                          "bitwise_not", gib, last=1)
    assert r["fetch_scale"] == pytest.approx(0.5)
    assert r["write_scale"] == pytest.approx(1.0)
    # the last dispatch only: 3000 KiB read at half scale, 30 KiB written
    assert r["fetch_bytes"] == pytest.approx(3000 * 1024 / 0.5)
    assert r["write_bytes"] == pytest.approx(30 * 1024)
    assert r["bytes_per_launch"] == pytest.approx(r["fetch_bytes"] + r["write_bytes"])


def test_trace_table_and_last_durations(tmp_path):
    p = tmp_path / "t.csv"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size", "VGPR_Count",
                    "Grid_Size_X", "Workgroup_Size_X"])
        w.writerow(["void ann::k_search<0, 8, 1, false, false>(ann::SearchArgs)", 0, 2_000_000, 0, 64, 640000, 64])
        w.writerow(["void ann::k_knn_mfma<2, 16>(unsigned char const*)", 2_000_000, 5_000_000, 52736, 100, 1, 256])
        w.writerow(["void ann::k_search<0, 8, 1, false, false>(ann::SearchArgs)", 5_000_000, 6_500_000, 0, 64,
                    640000, 64])
    table = profiling.trace_table(str(p))
    assert "`k_search<0, 8, 1, false, false>` | 2 | 1.750 | 3.5 |" in table
    assert "`k_knn_mfma<2, 16>` | 1 | 3.000 |" in table
    assert profiling.last_durations(str(p), r"k_search<0, 8, 1, false, false>", 1) == [1.5]


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    pkg = tmp_path / "pkg"
    for rel in profiling.KERNEL_SOURCES:
        os.makedirs(pkg / os.path.dirname(rel), exist_ok=True)
        shutil.copy(os.path.join(profiling.PKG, rel), pkg / rel)
    monkeypatch.setattr(profiling, "PKG", str(pkg))
    h0 = profiling.kernel_source_hash()
    assert len(h0) == 16 and int(h0, 16) >= 0
    src = pkg / profiling.KERNEL_SOURCES[0]
    text = src.read_text()
    src.write_text("// a new comment\n\n" + text.replace("\n", "  \n", 3) + "\n/* and a block\n comment */\n")
    assert profiling.kernel_source_hash() == h0
    src.write_text(text + "\nint extra_symbol;\n")
    assert profiling.kernel_source_hash() != h0


def test_traffic_record_is_read_only_on_matching_code(tmp_path, monkeypatch):
    md = tmp_path / "k_traffic.md"
    rec = '{"kernel": "k", "workload": "w T=1 nq=1", "bytes_per_launch": 5, "kernel_sources": "%s"}'
    md.write_text("text\n<!-- traffic-record " + rec % profiling.kernel_source_hash() + " -->\n")
    r = profiling.read_traffic_record(str(md))
    assert r is not None and r["bytes_per_launch"] == 5
    md.write_text("<!-- traffic-record " + rec % "0000000000000000" + " -->\n")
    assert profiling.read_traffic_record(str(md)) is None
    assert profiling.read_traffic_record(str(tmp_path / "absent.md")) is None


def test_algorithmic_bytes_counts_each_term():
    # columns: evals, ref pops, bridge pops, bridge ids, bridges extracted
    st = np.zeros((2, 12), np.int32)
    st[0, [0, 1, 3, 4]] = [1152, 191, 5, 4]
    st[1, [0, 1, 3, 4]] = [10, 0, 10, 32]
    b = bench.algorithmic_bytes(st, 128, 16, 10, 128)
    assert b[0] == 1152 * 128 + 191 * 4 * 16 + 4 * 8 + 5 * 4 + 128 + 80
    assert b[1] == 10 * 128 + 32 * 8 + 10 * 4 + 128 + 80


def test_bridge_alpha_counts_linked_vectors_per_bridge():
    off = np.array([0, 0, 3, 3, 4, 4, 4, 9], np.uint32)   # 7 bridges, 3 lists not empty
    ids = np.array([5, 1, 2, 5, 7, 8, 1, 9, 2], np.uint32)  # 6 distinct reference vectors
    idx = SimpleNamespace(export=lambda: {"bridge_off": off, "bridge_ids": ids})
    a = bench.bridge_alpha(idx)
    assert a["linked"] == 6
    assert a["alpha"] == pytest.approx(6 / 7)
    assert a["nonempty_share"] == pytest.approx(3 / 7)


def test_oracle_on_all_cores_matches_the_single_threaded_oracle():
    rng = np.random.default_rng(4)
    X = rng.integers(0, 256, (2000, 32), dtype=np.uint8)
    Q = rng.integers(0, 256, (40, 32), dtype=np.uint8)
    cb, g, off, ids = oracle.build_index(X, 2, 16, 8, 3, 1, 4, 5)
    parts = dict(codebooks=cb, graph=g, bridge_off=off, bridge_ids=ids)
    ref, _ = oracle.search(X, cb, g, off, ids, Q, 10, 150, 64)
    w = SimpleNamespace(k=10, queue_len=64)
    r = bench.oracle_all_cores(oracle, X, parts, Q, len(Q), 2, w, 150, ref)
    assert r["cores"] >= 1 and r["value"] > 0
    assert r["sample"].endswith("ids identical to the GPU: True")
    bad = ref.copy()
    bad[3, 0] = -5
    assert bench.oracle_all_cores(oracle, X, parts, Q, len(Q), 1, w, 150, bad)["sample"].endswith("False")
