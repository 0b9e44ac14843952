#!/usr/bin/env python3
"""Benchmark: delta-stepping SSSP on one MI355X.

Workload (default): directed R-MAT, scale 22 (4,194,304 vertices), edge factor 16,
(a, b, c, d) = (0.57, 0.19, 0.19, 0.05), vertex ids randomly permuted, uint32
weights uniform in [1, 255]; 64 random sources with out-edges. Delta is swept over
{8, 16, 32, 64, 128}; the timed steps use the fastest delta of the sweep.

One step = one pass over the 64 sources, each source one solver launch (the whole
hot path: split graph already resident, every bucket, light and heavy phase),
timed with HIP events on the launch stream. Inputs are resident in HBM before
the timed region. Per source the median over the timed steps is kept; `value`
is the harmonic mean over sources of GTEPS = m_reached / t, m_reached = out-edges
of reached vertices (the survey's protocol: warm-ups, median of 3, harmonic mean).
The same 64 sources solved in one launch (one after another on the whole device)
are reported beside it.

Beside the plain solve the line reports the batched and backward modes on the
same GPU ("modes"), each from the library's autotuner and timed with HIP events:
  concurrent_rmat_s22_k64  the plain workload with several sources in flight (concurrent groups)
  batched_rmat_s18_k256  R-MAT scale 18, fp32 log-uniform [1e-2, 1e2] weights, 256 sources:
                         concurrent sources in one cooperative launch replayed from a HIP
                         graph, against 256 looped single-source launches
  batched_ragged_er512   512 ER graphs (n log-uniform in [1e3, 1e5], degree 8, fp32 (0, 1])
                         as one block-diagonal graph, one source per block, solved at once
                         (nearest-source solve) from a HIP graph, against 512 per-graph solves
  backward_rmat_s18      R-MAT scale 18, fp32 [1, 2) weights, 16 sources, loss over 1024
                         targets: forward GTEPS and backward GTEPS = k * m / t_backward
  grid_4096              4096 x 4096 grid, u32 U[1, 1000], corner source, delta 50 / 100 / 400:
                         the high-diameter case (thousands of buckets), one source per launch

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "GTEPS & HBM GB/s, delta-stepping SSSP R-MAT s22; batched/backward vs plain"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_solver_rmat_s22.json")
CSRC = os.path.join(ROOT, "paper_1911_06895_amd", "csrc")


def kernel_source_hash() -> str:
    """Hash of the HIP sources: counter figures taken from another version are not reused."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(config_key: str):
    """HBM bytes per solver launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, scaled by the copy-kernel calibration -- or None when the summary is
    missing, was taken on another configuration, or the kernels changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("config_key") != config_key:
        return None
    return t["bytes_per_launch"]


def copy_calibration(gib: float, reps: int) -> None:
    """A plain device copy of known size, run under the same counters to scale them."""
    import torch

    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {reps} x {n * 4} bytes read and written")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _reached(row: np.ndarray) -> np.ndarray:
    return row != np.uint32(0xFFFFFFFF) if row.dtype == np.uint32 else np.isfinite(row)


def algorithmic_bytes(g, dist_rows: np.ndarray, improvements: int) -> float:
    """Lower bound on the bytes one solve must move (per source, summed):
    12 B per reached edge (8 B edge record + 4 B read of t[v]), 4 B per successful
    atomic update, 24 B per reached vertex (t[u] in the light and heavy phases,
    row offsets, frontier entry write and read)."""
    outdeg = g.outdeg()
    total = 0.0
    for row in np.atleast_2d(dist_rows):
        reached = _reached(row)
        total += 12.0 * float(outdeg[reached].sum()) + 24.0 * float(reached.sum())
    return total + 4.0 * float(improvements)


def adjoint_bytes(g, dist_rows: np.ndarray) -> float:
    """Lower bound on the bytes one adjoint launch moves: per source, the distance and coefficient
    rows (8 B per vertex), 12 B per reached edge (edge record + d(y) in the parent search) and 24 B
    per reached vertex (the parent record written and read, its fp64 coefficient); per launch,
    12 B per edge (the fp64 dL/dw accumulator read, the fp32 result written)."""
    outdeg = g.outdeg()
    total = 12.0 * g.m
    for row in np.atleast_2d(dist_rows):
        reached = _reached(row)
        total += 8.0 * g.n + 12.0 * float(outdeg[reached].sum()) + 24.0 * float(reached.sum())
    return total


def reached_edges(g, dist_rows: np.ndarray) -> int:
    outdeg = g.outdeg()
    return int(sum(int(outdeg[_reached(row)].sum()) for row in np.atleast_2d(dist_rows)))


def roof(bytes_per_launch: float, ms: float) -> dict:
    gbs = bytes_per_launch / ms / 1e6
    return {"algorithmic_gbs": round(gbs, 2), "hbm_frac": round(gbs / HBM_PEAK_GBS, 5)}


def cpu_baseline(g, sources, budget_s: float, gpu_rows: np.ndarray):
    """The CPU oracle (binary-heap Dijkstra, one core) on a bounded sample of the sources. The
    rows it computes are also compared with the GPU rows of the same sources (bit for bit)."""
    import oracle

    done, edges, t_total = 0, 0, 0.0
    for r, s in enumerate(sources):
        t0 = time.perf_counter()
        d, rc = oracle.dijkstra(g, int(s))
        dt = time.perf_counter() - t0
        if rc != oracle.OK:
            raise RuntimeError("oracle failed")
        if not np.array_equal(gpu_rows[r].view(np.uint32), d.view(np.uint32)):
            raise SystemExit(f"bench: GPU distances from source {s} differ from the oracle")
        t_total += dt
        edges += oracle.reached_edges(g, d)
        done += 1
        if t_total >= budget_s:
            break
    return {"value": edges / t_total / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{done} of {len(sources)} sources, binary-heap Dijkstra, single thread, "
                      f"{t_total:.1f} s (each row also matched the GPU row bit for bit)"}, done


def host_info() -> dict:
    """The host the CPU baselines ran on: logical CPUs, the CPUs this process may use, the model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_threads() -> int:
    """Threads for the multi-core baselines: the CPUs this process may use, at most 16 (the host
    share of one GPU)."""
    return max(1, min(16, host_info()["usable_cpus"]))


def cpu_baselines(g_c2, sources_c2, rows_c2, grid_row, threads: int) -> dict:
    """The oracle (binary-heap Dijkstra; the shortest-path-tree gradient for the backward workload),
    timed on the host outside every GPU timed region. Rows it computes are compared with the GPU's
    bit for bit. Single-thread figures run one solve at a time; the multi-core ones spread sources
    (or graphs) over `threads` host threads."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    from paper_1911_06895_amd import graphs as G

    out = {}
    # C2, every source, all cores
    t0 = time.perf_counter()
    d, rc = oracle.dijkstra_many(g_c2, sources_c2, threads)
    dt = time.perf_counter() - t0
    if rc != oracle.OK or not np.array_equal(d.view(np.uint32), rows_c2.view(np.uint32)):
        raise SystemExit("bench: the oracle's rows differ from the GPU's (R-MAT scale 22, 64 sources)")
    e = sum(oracle.reached_edges(g_c2, row) for row in d)
    out["rmat_s22_k64_all_cores"] = {"value": round(e / dt / 1e9, 4), "unit": "GTEPS", "cores": threads,
                                     "seconds": round(dt, 2), "sample": "all 64 sources, each row matched the GPU's"}
    del d
    # C1: mean of 100 runs, one core
    g1 = G.workload("er_n1024_m8192")
    t0 = time.perf_counter()
    for _ in range(100):
        d1, rc = oracle.dijkstra(g1, 0)
    dt = (time.perf_counter() - t0) / 100
    out["er_n1024_m8192"] = {"value": round(oracle.reached_edges(g1, d1) / dt / 1e9, 5), "unit": "GTEPS", "cores": 1,
                             "ms": round(dt * 1e3, 4), "sample": "source 0, mean of 100 runs"}
    # C3: one Dijkstra on the grid, one core (delta plays no part)
    if grid_row is not None:
        g3 = G.workload("grid4096_u32")
        t0 = time.perf_counter()
        d3, rc = oracle.dijkstra(g3, 0)
        dt = time.perf_counter() - t0
        if not np.array_equal(d3, grid_row):
            raise SystemExit("bench: the oracle's grid row differs from the GPU's")
        out["grid_4096"] = {"value": round(oracle.reached_edges(g3, d3) / dt / 1e9, 5), "unit": "GTEPS", "cores": 1,
                            "ms": round(dt * 1e3, 1), "sample": "corner source, one run, matched the GPU row"}
        del g3, d3
    # C4a: 256 sources of R-MAT scale 18 (fp32 log-uniform), source-parallel over all cores
    g4 = G.workload("rmat_s18_f32log")
    s4 = G.sources_with_outedges(g4, 256, cfg=41)
    t0 = time.perf_counter()
    d4, rc = oracle.dijkstra_many(g4, s4, threads)
    dt = time.perf_counter() - t0
    e = sum(oracle.reached_edges(g4, row) for row in d4)
    out["batched_rmat_s18_k256"] = {"value": round(e / dt / 1e9, 4), "unit": "GTEPS", "cores": threads,
                                    "ms": round(dt * 1e3, 1), "sample": "all 256 sources, source-parallel"}
    del d4
    # C4b: 512 ER graphs, graph-parallel over all cores
    graphs = G.ragged_er_batch(512, cfg=42)

    def one(gi):
        di, _ = oracle.dijkstra(gi, 0)
        return oracle.reached_edges(gi, di)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        e = sum(ex.map(one, graphs))
    dt = time.perf_counter() - t0
    out["batched_ragged_er512"] = {"value": round(e / dt / 1e9, 4), "unit": "GTEPS", "cores": threads,
                                   "ms": round(dt * 1e3, 1), "sample": "all 512 graphs, graph-parallel"}
    # C5: forward (16 Dijkstra) and the reference gradient, one core
    g5 = G.workload("rmat_s18_f32onetwo")
    s5 = G.sources_with_outedges(g5, 16, cfg=5)
    targets, coef = G.targets_and_coefs(g5.n, 1024, cfg=5)
    grad = np.zeros(g5.n)
    grad[targets] = coef
    acc = np.zeros(g5.m)
    t0 = time.perf_counter()
    rows = [oracle.dijkstra(g5, int(s))[0] for s in s5]
    tf = time.perf_counter() - t0
    for s, row in zip(s5, rows):
        oracle.sp_gradient(g5, int(s), row, np.where(np.isfinite(row), grad, 0.0), acc)
    tb = time.perf_counter() - t0 - tf
    e = sum(oracle.reached_edges(g5, row) for row in rows)
    out["backward_rmat_s18"] = {"forward_gteps": round(e / tf / 1e9, 4), "backward_gteps": round(16 * g5.m / tb / 1e9, 4),
                                "unit": "GTEPS", "cores": 1, "forward_ms": round(tf * 1e3, 1),
                                "backward_ms": round(tb * 1e3, 1),
                                "sample": "16 sources, 1024 targets: Dijkstra rows, then the tree gradient"}
    return out


def timed_ms(fn, reps: int = 1) -> float:
    """Mean device milliseconds of fn() on the current stream over reps calls, after one warm-up."""
    import torch

    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def device_graph(g, dev):
    import torch

    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col).to(dev)
    wt = torch.from_numpy(g.w.view(np.int32) if g.w.dtype == np.uint32 else g.w).to(dev)
    return rp, ci, wt


def captured(fn):
    """fn recorded into a HIP graph by stream capture; returns the replay callable."""
    import torch

    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        fn(stream)
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        fn(stream)
    return graph


def mode_concurrent_s22(g, sources, dev, steps: int, plain_rows: np.ndarray) -> dict:
    """The headline graph and sources with several sources in flight (concurrent groups), the
    delta and group count from the library's autotuner on 16 of the sources."""
    import torch

    from paper_1911_06895_amd import sssp

    rp, ci, wt = device_graph(g, dev)
    dist = torch.empty((len(sources), g.n), dtype=torch.int32, device=dev)
    h, tune = sssp.sssp_autotune(rp, ci, wt, sources[:16], dist[:16], deltas=[16, 32, 64, 128])
    src_dev = torch.from_numpy(np.asarray(sources, dtype=np.int32)).to(dev)
    ms = timed_ms(lambda: sssp.sssp_solve_async(h, src_dev, dist), reps=steps)
    sssp.sssp_solve_status(h)
    st = sssp.sssp_last_stats(h)
    tiles = sssp.sssp_get_tuning(h)
    rows = dist.cpu().numpy().view(np.uint32)
    sssp.sssp_destroy(h)
    if not np.array_equal(rows, plain_rows):
        raise SystemExit("bench: concurrent and one-at-a-time solves disagree")
    m_r = reached_edges(g, rows)
    return {"workload": "R-MAT scale 22 (the plain workload), 64 sources, several in flight",
            "delta": tune["delta"], "concurrent_sources": tune["concurrent_sources"], "tuning": tiles,
            "autotune_trials": tune["trials"], "ms": round(ms, 3), "gteps": round(m_r / ms / 1e6, 3),
            **roof(algorithmic_bytes(g, rows, st["improvements"]), ms)}


def mode_batched_s18(dev, steps: int) -> dict:
    import torch

    from paper_1911_06895_amd import graphs as G
    from paper_1911_06895_amd import sssp

    g = G.workload("rmat_s18_f32log")
    srcs = G.sources_with_outedges(g, 256, cfg=41)
    rp, ci, wt = device_graph(g, dev)
    dist = torch.empty((len(srcs), g.n), dtype=torch.float32, device=dev)
    h, tune = sssp.sssp_autotune(rp, ci, wt, srcs[:64], dist[:64])
    src_dev = torch.from_numpy(srcs).to(dev)
    graph = captured(lambda st: sssp.sssp_solve_async(h, src_dev, dist, st))
    ms = timed_ms(graph.replay, reps=steps)
    sssp.sssp_solve_status(h)
    st = sssp.sssp_last_stats(h)
    tiles = sssp.sssp_get_tuning(h)
    rows = dist.cpu().numpy()
    m_r = reached_edges(g, rows)
    b_alg = algorithmic_bytes(g, rows, st["improvements"])
    del graph
    sssp.sssp_destroy(h)
    # looped plain solves: one single-source launch per source, delta tuned for that on 16 sources
    one = dist[:1]
    best = None
    for delta in (0.5, 1.0, 2.0, 4.0, 8.0, 16.0):
        hd = sssp.sssp_create(rp, ci, wt, delta)
        t = timed_ms(lambda: [sssp.sssp_solve_async(hd, src_dev[r:r + 1], one) for r in range(16)])
        sssp.sssp_solve_status(hd)
        if best is None or t < best[1]:
            if best is not None:
                sssp.sssp_destroy(best[0])
            best = (hd, t, delta)
        else:
            sssp.sssp_destroy(hd)
    hl, _, dl = best
    outs = [dist[r:r + 1] for r in range(len(srcs))]
    ms_loop = timed_ms(lambda: [sssp.sssp_solve_async(hl, src_dev[r:r + 1], outs[r]) for r in range(len(srcs))])
    sssp.sssp_solve_status(hl)
    sssp.sssp_destroy(hl)
    if not np.array_equal(dist.cpu().numpy().view(np.uint32), rows.view(np.uint32)):
        raise SystemExit("bench: batched and looped solves disagree")
    return {"workload": "R-MAT scale 18 edge factor 16, fp32 log-uniform [1e-2,1e2], 256 sources",
            "n": g.n, "m": g.m, "m_reached": m_r, "delta": tune["delta"],
            "concurrent_sources": tune["concurrent_sources"], "tuning": tiles, "autotune_trials": tune["trials"],
            "ms": round(ms, 3), "gteps": round(m_r / ms / 1e6, 3), **roof(b_alg, ms),
            "looped": {"delta": dl, "ms": round(ms_loop, 3), "gteps": round(m_r / ms_loop / 1e6, 3)},
            "speedup_vs_looped": round(ms_loop / ms, 2), "hip_graph": True}


def mode_batched_ragged(dev, steps: int) -> dict:
    import torch

    from paper_1911_06895_amd import graphs as G
    from paper_1911_06895_amd import sssp

    graphs = G.ragged_er_batch(512, cfg=42)
    u, offs = G.block_union(graphs)
    rp, ci, wt = device_graph(u, dev)
    dist = torch.empty(u.n, dtype=torch.float32, device=dev)
    starts = offs[:-1].astype(np.int32)
    h, tune = sssp.sssp_autotune(rp, ci, wt, starts, dist, multi=True)
    src_dev = torch.from_numpy(starts).to(dev)
    graph = captured(lambda st: sssp.sssp_solve_multi_async(h, src_dev, dist, st))
    ms = timed_ms(graph.replay, reps=steps)
    sssp.sssp_solve_status(h)
    st = sssp.sssp_last_stats(h)
    tiles = sssp.sssp_get_tuning(h)
    d = dist.cpu().numpy()
    m_r = int(u.outdeg()[np.isfinite(d)].sum())
    b_alg = algorithmic_bytes(u, d, st["improvements"])
    del graph
    sssp.sssp_destroy(h)
    # looped plain solves: one handle and one single-source launch per graph, same delta
    handles, outs = [], []
    zero = torch.zeros(1, dtype=torch.int32, device=dev)
    for gi in graphs:
        handles.append(sssp.sssp_create(*device_graph(gi, dev), tune["delta"]))
        outs.append(torch.empty(gi.n, dtype=torch.float32, device=dev))
    ms_loop = timed_ms(lambda: [sssp.sssp_solve_async(hh, zero, o) for hh, o in zip(handles, outs)])
    for hh in handles:
        sssp.sssp_solve_status(hh)
        sssp.sssp_destroy(hh)
    if not np.array_equal(np.concatenate([o.cpu().numpy() for o in outs]).view(np.uint32), d.view(np.uint32)):
        raise SystemExit("bench: batched and per-graph solves disagree")
    return {"workload": "512 directed ER graphs, n log-uniform [1e3,1e5], m = 8n, fp32 (0,1], source 0 of each",
            "n": u.n, "m": u.m, "m_reached": m_r, "delta": tune["delta"], "tuning": tiles,
            "autotune_trials": tune["trials"], "ms": round(ms, 3), "gteps": round(m_r / ms / 1e6, 3),
            **roof(b_alg, ms),
            "looped": {"delta": tune["delta"], "ms": round(ms_loop, 3), "gteps": round(m_r / ms_loop / 1e6, 3)},
            "speedup_vs_looped": round(ms_loop / ms, 2), "hip_graph": True}


def mode_backward(dev, steps: int) -> dict:
    import torch

    from paper_1911_06895_amd import graphs as G
    from paper_1911_06895_amd import sssp

    g = G.workload("rmat_s18_f32onetwo")
    srcs = G.sources_with_outedges(g, 16, cfg=5)
    targets, coef = G.targets_and_coefs(g.n, 1024, cfg=5)
    rp, ci, wt = device_graph(g, dev)
    dist = torch.empty((len(srcs), g.n), dtype=torch.float32, device=dev)
    h, tune = sssp.sssp_autotune(rp, ci, wt, srcs, dist)
    grad_rows = np.zeros((len(srcs), g.n), dtype=np.float32)
    grad_rows[:, targets] = coef
    gd = torch.from_numpy(grad_rows).to(dev)
    gw = torch.empty(g.m, dtype=torch.float32, device=dev)
    ms_f = timed_ms(lambda: sssp.sssp_solve(h, srcs, dist), reps=steps)
    st = sssp.sssp_last_stats(h)
    ms_b = timed_ms(lambda: sssp.sssp_backward(h, srcs, dist, gd, gw), reps=steps)
    tiles = sssp.sssp_get_tuning(h)
    d = dist.cpu().numpy()
    m_r = reached_edges(g, d)
    sssp.sssp_destroy(h)
    fwd, bwd = roof(algorithmic_bytes(g, d, st["improvements"]), ms_f), roof(adjoint_bytes(g, d), ms_b)
    return {"workload": "R-MAT scale 18 edge factor 16, fp32 [1,2), 16 sources, 1024 targets, c ~ N(0,1)",
            "n": g.n, "m": g.m, "m_reached": m_r, "delta": tune["delta"],
            "concurrent_sources": tune["concurrent_sources"], "tuning": tiles,
            "forward_ms": round(ms_f, 3), "forward_gteps": round(m_r / ms_f / 1e6, 3),
            "forward_algorithmic_gbs": fwd["algorithmic_gbs"], "forward_hbm_frac": fwd["hbm_frac"],
            "backward_ms": round(ms_b, 3), "backward_gteps": round(len(srcs) * g.m / ms_b / 1e6, 3),
            "backward_algorithmic_gbs": bwd["algorithmic_gbs"], "backward_hbm_frac": bwd["hbm_frac"]}


def mode_grid(dev, steps: int) -> dict:
    """The high-diameter workload: a 4096 x 4096 4-neighbour grid, u32 weights U[1,1000] per
    directed edge, the corner source, one source per launch, for each delta of {50, 100, 400}.
    Thousands of buckets with small frontiers: bound by the latency of the steps and their
    barriers rather than by HBM, which the per-phase time and the algorithmic GB/s show."""
    import torch

    from paper_1911_06895_amd import graphs as G
    from paper_1911_06895_amd import sssp

    g = G.workload("grid4096_u32")
    rp, ci, wt = device_graph(g, dev)
    src = np.zeros(1, dtype=np.int32)
    dist = torch.empty((1, g.n), dtype=torch.int32, device=dev)
    per_delta, ref = {}, None
    for delta in (50.0, 100.0, 400.0):
        h = sssp.sssp_create(rp, ci, wt, delta)
        ms = timed_ms(lambda: sssp.sssp_solve(h, src, dist), reps=steps)
        st = sssp.sssp_last_stats(h)
        sssp.sssp_destroy(h)
        rows = dist.cpu().numpy().view(np.uint32)
        if ref is None:
            ref = rows.copy()
        elif not np.array_equal(rows, ref):
            raise SystemExit("bench: grid distances differ between deltas")
        m_r = reached_edges(g, rows)
        gbs = algorithmic_bytes(g, rows, st["improvements"]) / ms / 1e6
        phases = st["light_phases"] + st["heavy_phases"]
        per_delta[f"{delta:g}"] = {"ms": round(ms, 3), "gteps": round(m_r / ms / 1e6, 4),
                                   "algorithmic_gbs": round(gbs, 2), "hbm_frac": round(gbs / HBM_PEAK_GBS, 5),
                                   "buckets": st["buckets"], "phases": phases,
                                   "us_per_phase": round(ms * 1e3 / max(1, phases), 2)}
    best = min(per_delta, key=lambda k: per_delta[k]["ms"])
    GRID_ROW["row"] = ref[0]
    return {"workload": "grid 4096 x 4096, 4-neighbour, u32 U[1,1000], corner source, one source per launch",
            "n": g.n, "m": g.m, "best_delta": float(best), "per_delta": per_delta}


GRID_ROW = {"row": None}  # the grid's GPU distances, compared with the oracle's in the CPU baselines


def per_source_times(handle, sources, dist, stream, passes: int) -> np.ndarray:
    """`passes` passes over the sources, each source one launch (sssp_solve_async on a device
    source) bracketed by HIP events on the launch stream; returns milliseconds [passes, k]."""
    import torch

    from paper_1911_06895_amd import sssp

    k = len(sources)
    src_dev = torch.from_numpy(np.asarray(sources, dtype=np.int32)).to(dist.device)
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
          for _ in range(passes)]
    for p in range(passes):
        for r in range(k):
            ev[p][r][0].record(stream)
            sssp.sssp_solve_async(handle, src_dev[r:r + 1], dist[r:r + 1], stream)
            ev[p][r][1].record(stream)
    torch.cuda.synchronize()
    sssp.sssp_solve_status(handle, stream)
    return np.array([[ev[p][r][0].elapsed_time(ev[p][r][1]) for r in range(k)] for p in range(passes)])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed passes over the sources (median per source)")
    ap.add_argument("--warmup", type=int, default=3, help="untimed passes over the sources")
    ap.add_argument("--workload", default="rmat_s22_u32")
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--deltas", default="8,16,32,64,128")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of single-core oracle time (headline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true", help="only the plain R-MAT scale 22 solve")
    ap.add_argument("--only", default="", help="run only this mode (concurrent, batched, ragged, backward, grid) "
                                               "after the plain solve, for per-mode profiles")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of this many GiB (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1911_06895_amd import graphs as G
    from paper_1911_06895_amd import sssp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration, 5)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.perf_counter()
    g = G.workload(args.workload)
    sources = G.sources_with_outedges(g, args.sources, cfg=2)
    log(f"[bench] graph {args.workload}: n={g.n} m={g.m} generated in {time.perf_counter() - t0:.1f}s")

    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col).to(dev)
    wt = torch.from_numpy(g.w.view(np.int32) if g.w.dtype == np.uint32 else g.w).to(dev)
    out_dtype = torch.int32 if g.w.dtype == np.uint32 else torch.float32
    dist = torch.empty((len(sources), g.n), dtype=out_dtype, device=dev)
    stream = torch.cuda.current_stream()

    def run(handle):
        sssp.sssp_solve(handle, sources, dist, stream)

    def host_rows():
        return dist.cpu().numpy().view(np.uint32) if out_dtype == torch.int32 else dist.cpu().numpy()

    # delta sweep: create (split) + one warm solve + one timed solve of all sources in one launch per delta
    sweep = {}
    best = None
    for delta in [float(x) for x in args.deltas.split(",")]:
        tc = time.perf_counter()
        h = sssp.sssp_create(rp, ci, wt, delta, stream)
        torch.cuda.synchronize()
        t_create = time.perf_counter() - tc
        run(h)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run(h)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        m_r = reached_edges(g, host_rows())
        st = sssp.sssp_last_stats(h)
        gteps = m_r / (ms * 1e-3) / 1e9
        sweep[str(int(delta) if delta.is_integer() else delta)] = {
            "gteps": round(gteps, 3), "ms_per_source": round(ms / len(sources), 4), "create_ms": round(t_create * 1e3, 2),
            "buckets_per_source": round(st["buckets"] / len(sources), 1),
            "phases_per_source": round((st["light_phases"] + st["heavy_phases"]) / len(sources), 1)}
        log(f"[bench] delta={delta:g}: {gteps:.2f} GTEPS, {ms / len(sources):.3f} ms/source, "
            f"create {t_create * 1e3:.1f} ms, stats {st}")
        if best is None or gteps > best[1]:
            if best is not None:
                sssp.sssp_destroy(best[0])
            best = (h, gteps, delta)
        else:
            sssp.sssp_destroy(h)
    handle, _, delta = best

    # the same sources in one launch (one after another on the whole device): its rows are checked
    # by sssp_solve's status and against the oracle below; its counters give the atomic updates
    run(handle)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        run(handle)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_one_launch = e0.elapsed_time(e1) / args.steps
    st = sssp.sssp_last_stats(handle)
    tuning_main = sssp.sssp_get_tuning(handle)  # the handle is released before the modes run
    rows = host_rows()
    m_rows = np.array([reached_edges(g, row) for row in rows], dtype=np.float64)
    b_rows = np.array([algorithmic_bytes(g, row, 0) for row in rows]) + 4.0 * st["improvements"] / len(sources)

    # the timed region: `steps` passes over the sources, one launch per source, after `warmup` passes
    if args.warmup > 0:
        per_source_times(handle, sources, dist, stream, args.warmup)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    times = per_source_times(handle, sources, dist, stream, args.steps)
    t_wall = time.perf_counter() - t_wall
    if not np.array_equal(host_rows(), rows):
        raise SystemExit("bench: per-source launches and the one-launch solve disagree")
    med = np.median(times, axis=0)  # ms per source
    gteps_rows = m_rows / (med * 1e-3) / 1e9
    value = len(sources) / float(np.sum(1.0 / gteps_rows))  # harmonic mean over sources
    ms_step = float(np.mean(times.sum(axis=1)))
    achieved = float(b_rows.sum()) / (float(med.sum()) * 1e-3) / 1e9
    log(f"[bench] timed: delta={delta:g}, {args.steps} passes of {len(sources)} launches, {med.mean():.3f} ms per "
        f"source (median of {args.steps}), {value:.2f} GTEPS (harmonic mean), algorithmic {achieved:.1f} GB/s; "
        f"one launch of all sources {ms_one_launch:.2f} ms; wall {t_wall:.2f} s")

    modes = {}
    want = (lambda name: not args.no_modes and (not args.only or args.only == name))
    if want("concurrent") and args.workload == "rmat_s22_u32":
        t0 = time.perf_counter()
        del dist
        sssp.sssp_destroy(handle)
        handle = None
        torch.cuda.empty_cache()
        modes["concurrent_rmat_s22_k64"] = mode_concurrent_s22(g, sources, dev, max(1, args.steps), rows)
        log(f"[bench] concurrent_rmat_s22_k64: {modes['concurrent_rmat_s22_k64']} ({time.perf_counter() - t0:.1f}s)")
    for key, name, fn in (("batched", "batched_rmat_s18_k256", mode_batched_s18),
                          ("ragged", "batched_ragged_er512", mode_batched_ragged),
                          ("backward", "backward_rmat_s18", mode_backward), ("grid", "grid_4096", mode_grid)):
        if want(key):
            t0 = time.perf_counter()
            modes[name] = fn(dev, max(1, args.steps))
            log(f"[bench] {name}: {modes[name]} ({time.perf_counter() - t0:.1f}s)")
            torch.cuda.empty_cache()

    cpu, checked, others = None, 0, None
    if not args.no_cpu_baseline:
        cpu, checked = cpu_baseline(g, sources, args.cpu_budget, rows)
        cpu["host"] = host_info()
        log(f"[bench] cpu baseline: {cpu}")
        if not args.no_modes and not args.only and args.workload == "rmat_s22_u32":
            others = cpu_baselines(g, sources, rows, GRID_ROW["row"], cpu_threads())
            log(f"[bench] cpu baselines: {others}")

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if g.w.dtype == np.uint32 else "f32",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale 22 edge factor 16 (a,b,c,d)=(0.57,0.19,0.19,0.05) permuted, "
                               f"u32 weights U[1,255]" if args.workload == "rmat_s22_u32" else args.workload,
                   "n": g.n, "m": g.m, "sources": len(sources), "delta": delta, "m_reached": int(m_rows.sum()),
                   "protocol": f"one launch per source, HIP events on the launch stream, {args.warmup} warm-up and "
                               f"{args.steps} timed passes, median per source, harmonic mean of GTEPS",
                   "ms_per_source_mean": round(float(med.mean()), 4),
                   "gteps_min_max": [round(float(gteps_rows.min()), 3), round(float(gteps_rows.max()), 3)],
                   "one_launch_all_sources": {"ms": round(ms_one_launch, 3),
                                              "gteps": round(float(m_rows.sum()) / ms_one_launch / 1e6, 3)},
                   "tuning": tuning_main,
                   "delta_sweep": sweep, "oracle_checked_sources": checked},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": measured_traffic(f"{args.workload}:k1:delta{delta:g}")},
        "cpu_baseline": cpu,
        "cpu_baselines": others,
        "modes": modes,
    }
    print(json.dumps(out), flush=True)
    # release everything explicitly before the interpreter exits: handles, tensors, the device
    if handle is not None:
        sssp.sssp_destroy(handle)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    sys.stdout.flush()
    sys.stderr.flush()


if __name__ == "__main__":
    main()
