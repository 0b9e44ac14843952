"""Host-side arithmetic of bench.py (no GPU): the reached-edge count behind
GTEPS, the algorithmic-bytes formula behind the roofline figure, the traffic
record's guard against stale counters, and the refusal of several GPUs."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
from paper_1911_06895_amd.graphs import Graph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INF32 = np.uint32(0xFFFFFFFF)


def tiny_graph(wdtype=np.uint32):
    # 0 -> 1, 0 -> 2, 1 -> 2, 3 -> 0, 3 -> 1: from source 0, vertex 3 is never reached
    row_ptr = np.array([0, 2, 3, 3, 5], dtype=np.int64)
    col = np.array([1, 2, 2, 0, 1], dtype=np.int32)
    w = np.array([3, 9, 4, 1, 1], dtype=wdtype)
    return Graph(4, row_ptr, col, w)


def test_reached_edges_counts_out_edges_of_reached_vertices():
    g = tiny_graph()
    rows = np.array([[0, 3, 7, INF32], [INF32, INF32, INF32, 0]], dtype=np.uint32)
    # row 0 reaches 0, 1, 2 (out-degrees 2, 1, 0); row 1 reaches only 3 (out-degree 2)
    assert bench.reached_edges(g, rows) == 3 + 2
    gf = tiny_graph(np.float32)
    rows_f = np.array([[0.0, 3.0, 7.0, np.inf]], dtype=np.float32)
    assert bench.reached_edges(gf, rows_f) == 3


def test_algorithmic_bytes_follow_the_stated_formula():
    """12 B per reached edge, 24 B per reached vertex, 4 B per successful atomic update."""
    g = tiny_graph()
    rows = np.array([[0, 3, 7, INF32], [INF32, INF32, INF32, 0]], dtype=np.uint32)
    improvements = 5
    want = 12 * (3 + 2) + 24 * (3 + 1) + 4 * improvements
    assert bench.algorithmic_bytes(g, rows, improvements) == want


def test_traffic_record_is_ignored_for_other_sources_or_configurations(tmp_path, monkeypatch):
    rec = {"config_key": "rmat_s22_u32:k64:delta64", "kernel_source_hash": bench.kernel_source_hash(),
           "bytes_per_launch": 123}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("rmat_s22_u32:k64:delta64") == 123
    assert bench.measured_traffic("rmat_s22_u32:k64:delta32") is None  # another delta
    rec["kernel_source_hash"] = "0" * 16  # counters taken from other kernel sources
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("rmat_s22_u32:k64:delta64") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("rmat_s22_u32:k64:delta64") is None


def test_kernel_source_hash_covers_the_hip_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert any(f.endswith(".hip") for f in os.listdir(bench.CSRC))


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
