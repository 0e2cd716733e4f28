"""Host-side tooling the measurements rest on (no GPU): the benchmark's
one-GPU contract, its algorithmic-byte model, and the rocprofv3 summary
tools (copy calibration of the traffic counters, the stale-source check)."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1805_04207_amd import profile_summary as ps  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_bytes_model():
    n_ev, n_wi, n_mem, n_br = 1000, 10, 300, 50
    ab = lambda k, p=2: bench.algorithmic_bytes(k, n_ev, n_wi, n_mem, n_br, p)
    assert ab("k_ops") == 2 * n_ev + 8 * (n_wi + 1)
    assert ab("k_mem_bucket") == 8 * n_mem
    assert ab("k_mem_scatter") == ab("k_mem_hist") + 8 * n_mem
    assert ab("k_br_sort", 2) == 2 * ab("k_br_sort", 1)
    assert ab("k_finalize") == 0.0
    assert set(bench.MAIN_STREAM_KERNELS) >= {"k_mem_bucket", "k_mem_scatter", "k_finalize"}


def _db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, "
                "value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_is_scaled_by_the_calibration_copy(tmp_path):
    copy = 1 << 20                                  # bytes the calibration copy moves
    k = "void (anonymous namespace)::k_mem_bucket<false>(TraceArgs, TraceArgs const*)"
    # the counter reads half the copy's bytes (KiB): scale 2; writes read in full
    _db(tmp_path / "f.db", [(k, "FETCH_SIZE", 3000.0), (k, "FETCH_SIZE", 5000.0),
                            ("__amd_rocclr_copyBuffer", "FETCH_SIZE", copy / 2048.0),
                            ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 1.0)])
    _db(tmp_path / "w.db", [(k, "WRITE_SIZE", 10.0),
                            ("__amd_rocclr_copyBuffer", "WRITE_SIZE", copy / 1024.0)])
    out = tmp_path / "traffic.md"

    class A:
        fetch_db, write_db = str(tmp_path / "f.db"), str(tmp_path / "w.db")
        kernel, workload, copy_bytes, cmd, o = "k_mem_bucket", "w1", copy, "cmd", str(out)
    assert ps.traffic(A) == 0
    rec = ps.read_traffic(str(out), "k_mem_bucket", "w1")
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["fetch_bytes"] == pytest.approx(4000.0 * 1024 * 2)   # mean of two dispatches
    assert rec["write_bytes"] == pytest.approx(10.0 * 1024)
    assert ps.read_traffic(str(out), "k_mem_bucket", "another workload") is None
    # a record from other kernel sources is not reported
    text = out.read_text().replace(rec["sources"], "0" * 16)
    out.write_text(text)
    assert ps.read_traffic(str(out), "k_mem_bucket", "w1") is None


def test_source_hash_of_one_kernel_ignores_other_sources():
    full, one = ps.sources_hash(), ps.sources_hash("k_mem_bucket")
    assert full != one and len(one) == 16
    assert ps.sources_hash("k_mem_bucket") == one
