"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Distances are unique (the minimum over paths of a fold that is monotone and
non-decreasing), so every comparison is bit-exact: uint32 for integer weights
and 0 ulp for fp32 weights. A nonzero fp32 difference would be reported with
its size; the allowed relative tolerance 1e-6 is never used because none is seen.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1911_06895_amd import graphs as G  # noqa: E402
from paper_1911_06895_amd import sssp  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU-only hosts
    pytest.skip("no GPU", allow_module_level=True)


def _bits(a):
    if a.dtype == np.float32:
        return a.view(np.uint32)
    if a.dtype == np.float64:
        return a.view(np.uint64)
    return a


def gpu_solve(g, delta, sources, tuning=None):
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, delta)
    try:
        if tuning:
            solver.set_tuning(**tuning)
        d = solver.solve_numpy(sources)
        return d, solver.stats()
    finally:
        solver.close()


def assert_exact(g, got, src, label=""):
    want, rc = oracle.dijkstra(g, int(src))
    assert rc == oracle.OK
    if not np.array_equal(_bits(got), _bits(want)):
        bad = np.nonzero(_bits(got) != _bits(want))[0]
        detail = ""
        if got.dtype == np.float32:
            fin = np.isfinite(want[bad]) & np.isfinite(got[bad])
            rel = np.abs(got[bad][fin].astype(np.float64) - want[bad][fin]) / np.maximum(want[bad][fin], 1e-30)
            detail = f" max rel diff {rel.max() if rel.size else 'n/a'}"
        raise AssertionError(f"{label} source {src}: {bad.size} vertices differ, first {bad[:5]}: "
                             f"got {got[bad[:5]]} want {want[bad[:5]]}{detail}")


def certify_rows(g, srcs, rows, label=""):
    """Every row through the oracle's O(m) optimality certificate, on host threads."""
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        codes = list(ex.map(lambda r: oracle.certify(g, int(srcs[r]), rows[r]), range(len(srcs))))
    bad = [(r, c) for r, c in enumerate(codes) if c != oracle.CERT_OK]
    assert not bad, f"{label}: rows not certified (row, code): {bad[:8]}"


def test_er_1024_all_deltas():
    g = G.workload("er_n1024_m8192")
    for delta in (1, 8, 32, 100, 1000, 100000):
        got, st = gpu_solve(g, delta, [0])
        assert_exact(g, got[0], 0, f"delta={delta}")
        assert st["sources"] == 1


def test_multi_source_rows():
    g = G.workload("er_n1024_m8192")
    srcs = [0, 5, 1023, 512, 5]
    got, st = gpu_solve(g, 32, srcs)
    for r, s in enumerate(srcs):
        assert_exact(g, got[r], s)
    assert st["sources"] == len(srcs)


@pytest.mark.parametrize("wkind", ["u32", "f32", "f64"])
def test_sources_without_in_edges(wkind):
    """Vertices without in-edges are reached only as seeds (the output copy gives the others
    infinity without reading their distance): a source with no in-edges, a row whose source has
    in-edges, rows of invalid sources, and a nearest-source solve whose seeds have no in-edges."""
    r = G.rng_for(77, G.S_STRUCT)
    n, m = 3000, 9000
    src = r.integers(0, n // 2, size=m)          # in-edges only into the upper half, out-edges from
    dst = r.integers(n // 3, n, size=m)          # the lower half: many vertices have no in-edges
    w = {"u32": r.integers(1, 100, size=m).astype(np.uint32),
         "f32": r.uniform(0.5, 4.0, size=m).astype(np.float32),
         "f64": r.uniform(0.5, 4.0, size=m)}[wkind]
    g = G.csr_from_edges(n, src, dst, w)
    indeg = np.bincount(g.col, minlength=n)
    outdeg = np.diff(g.row_ptr)
    no_in = np.nonzero((indeg == 0) & (outdeg > 0))[0]
    with_in = np.nonzero((indeg > 0) & (outdeg > 0))[0]
    assert no_in.size > 10 and with_in.size > 10
    srcs = [int(no_in[0]), int(with_in[0]), int(no_in[-1])]
    got, _ = gpu_solve(g, 8.0, srcs)
    for row, s0 in enumerate(srcs):
        assert_exact(g, got[row], s0, f"{wkind} no-in-edges")
        assert got[row][s0] == 0
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 8.0)
    try:
        seeds = [int(x) for x in no_in[:5]]
        d = solver.solve_multi(seeds).cpu().numpy()
        if d.dtype == np.int32:  # u32 distances come back in an int32 tensor
            d = d.view(np.uint32)
        want = np.stack([oracle.dijkstra(g, x)[0] for x in seeds]).min(axis=0)
        assert np.array_equal(_bits(d), _bits(want))
        assert all(d[x] == 0 for x in seeds)
    finally:
        solver.close()


@pytest.mark.parametrize("seed", range(12))
def test_random_graphs_ragged(seed):
    """Sizes that span several 256-entry tiles with a ragged tail, raw CSR (parallel
    edges and self-loops kept), both weight types."""
    r = G.rng_for(9000 + seed, G.S_STRUCT)
    n = int(r.integers(300, 5000))
    m = int(r.integers(n, 12 * n))
    src = r.integers(0, n, size=m)
    dst = r.integers(0, n, size=m)
    if seed % 2 == 0:
        w = r.integers(1, 1000, size=m).astype(np.uint32)
        deltas = [1, 37, 256, 5000]
    else:
        w = np.exp(r.uniform(np.log(1e-2), np.log(1e2), size=m)).astype(np.float32)
        deltas = [0.25, 1.0, 3.3, 0.07]  # two dyadic, two not (fp32 re-insertion path)
    g = G.csr_from_edges(n, src, dst, w, dedup=seed % 3 != 0, drop_self_loops=seed % 3 != 0)
    s = int(G.sources_with_outedges(g, 1, cfg=9000 + seed)[0])
    for delta in deltas:
        got, _ = gpu_solve(g, delta, [s])
        assert_exact(g, got[0], s, f"seed={seed} delta={delta}")


@pytest.mark.parametrize("delta", [8, 32, 128])
def test_rmat_s14(delta):
    g = G.rmat_graph(14, 16, cfg=2)
    srcs = G.sources_with_outedges(g, 3, cfg=2)
    got, st = gpu_solve(g, delta, srcs)
    for r, s in enumerate(srcs):
        assert_exact(g, got[r], s, f"rmat14 delta={delta}")
    # each reached heavy edge is relaxed exactly once per solve (schedule invariant)
    heavy = 0
    light = 0
    for r, s in enumerate(srcs):
        reached = got[r] != 0xFFFFFFFF
        src_of_edge = g.edge_src()
        mask = reached[src_of_edge]
        heavy += int((mask & (g.w > delta)).sum())
        light += int((mask & (g.w <= delta)).sum())
    assert st["heavy_edges"] == heavy
    assert st["light_edges"] >= light


def _heavy_phase_records(g, delta, src, tuning=None):
    """(bucket, input entries) of every heavy phase of one traced solve: the input of bucket i's
    heavy phase is S_i, the vertices expanded in bucket i (Sec. IV-D)."""
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, delta)
    try:
        if tuning:
            solver.set_tuning(**tuning)
        cap = 1 << 16
        buf = torch.zeros(4 * cap, dtype=torch.int64, device="cuda")
        sssp.sssp_set_trace(solver.handle, buf, cap)
        d = solver.solve_numpy([src])[0]
        st = solver.stats()
        sssp.sssp_set_trace(solver.handle, None, 0)
        words = buf.cpu().numpy().view(np.uint64).reshape(-1, 4)[:min(cap, st["trace_records"])]
    finally:
        solver.close()
    assert st["trace_records"] <= cap
    what = words[:, 1]
    action = (what & np.uint64(0x7F)).astype(np.int64)
    bucket = ((what >> np.uint64(8)) & np.uint64(0xFFFFFF)).astype(np.int64)
    entries = (what >> np.uint64(32)).astype(np.int64)
    heavy = action == 2
    return d, bucket[heavy], entries[heavy]


@pytest.mark.parametrize("kind,delta,chain", [("rmat", 8, 0), ("rmat", 32, 0), ("rmat", 128, 0), ("grid", 50, 0),
                                              ("er", 16, 0), ("rmat", 32, 1), ("er", 16, 1), ("grid", 50, 2)])
def test_bucket_schedule_matches_oracle_trace(kind, delta, chain):
    """Schedule invariants of Fig. 1 on the GPU (integer weights, where no bucket is repeated):
    the non-empty buckets and each |S_i| equal those of the oracle's literal linear-algebra run,
    and S_i = {v : floor(d(v) / delta) = i}; with the library's default for the graph (chain 0),
    and with the leader's chained light steps forced on (1) or off (2)."""
    if kind == "rmat":
        g = G.rmat_graph(14, 16, cfg=2)
    elif kind == "grid":
        g = G.grid_graph(64, 64, cfg=3)
    else:
        g = G.workload("er_n1024_m8192")
    src = int(G.sources_with_outedges(g, 1, cfg=7)[0])
    d, buckets, sizes = _heavy_phase_records(g, delta, src, {"leader_chain": chain} if chain else None)
    want_d, rc, tr = oracle.delta_stepping_la(g, delta, src)
    assert rc == oracle.OK and np.array_equal(d, want_d)
    nz = sizes > 0  # a bucket whose ring slot held only vertices that had moved lower expands nothing
    assert np.array_equal(buckets[nz], tr["buckets"]), "non-empty buckets differ from the oracle trace"
    assert np.array_equal(sizes[nz], tr["s_size"]), "|S_i| differs from the oracle trace"
    fin = d != np.uint32(0xFFFFFFFF)
    by_dist = np.bincount((d[fin] // delta).astype(np.int64))
    assert np.array_equal(np.nonzero(by_dist)[0], tr["buckets"])
    assert np.array_equal(by_dist[by_dist > 0], sizes[nz])


def test_grid_many_buckets():
    g = G.grid_graph(96, 96, cfg=3)
    for delta in (50, 400):
        got, st = gpu_solve(g, delta, [0])
        assert_exact(g, got[0], 0, f"grid delta={delta}")
        assert st["buckets"] >= len(np.unique(got[0] // delta))


def test_far_list_path():
    """Weights far larger than delta: the near ring (64 buckets) overflows into the far list."""
    r = G.rng_for(9100, G.S_STRUCT)
    n, m = 3000, 24000
    g = G.csr_from_edges(n, r.integers(0, n, m), r.integers(0, n, m), r.integers(1, 10**6, m).astype(np.uint32))
    got, st = gpu_solve(g, 1000, [7])
    assert_exact(g, got[0], 7, "far")
    assert st["far_phases"] > 0


def test_fp32_loguniform_rmat():
    g = G.rmat_graph(13, 16, cfg=41, weights="f32_loguniform", wlo=1e-2, whi=1e2)
    srcs = G.sources_with_outedges(g, 2, cfg=41)
    for delta in (0.5, 2.0, 0.3):
        got, _ = gpu_solve(g, delta, srcs)
        for r, s in enumerate(srcs):
            assert_exact(g, got[r], s, f"f32 delta={delta}")


def test_fp32_absorption_golden():
    """The fp32 worked example: 2^24 + 1 rounds to 2^24 along the two-hop path."""
    g = G.csr_from_edges(4, np.array([0, 1, 0, 2]), np.array([1, 2, 2, 3]),
                         np.array([16777216.0, 1.0, 16777218.0, 2.0], dtype=np.float32), dedup=False)
    got, _ = gpu_solve(g, 4.0, [0])
    assert np.array_equal(got[0], np.array([0.0, 16777216.0, 16777216.0, 16777218.0], dtype=np.float32))


def test_edge_cases():
    # single vertex, no edges
    g = G.Graph(n=1, row_ptr=np.zeros(2, dtype=np.int64), col=np.zeros(0, dtype=np.int32),
                w=np.zeros(0, dtype=np.uint32))
    got, st = gpu_solve(g, 5, [0])
    assert got[0].tolist() == [0]
    # source without out-edges: everything else unreachable
    g = G.path_graph(50, np.arange(1, 50, dtype=np.uint32))
    got, _ = gpu_solve(g, 3, [49])
    assert got[0][49] == 0 and np.all(got[0][:49] == 0xFFFFFFFF)
    got, _ = gpu_solve(g, 3, [0])
    assert np.array_equal(got[0], np.concatenate([[0], np.cumsum(np.arange(1, 50))]).astype(np.uint32))
    # largest representable distance 2^32 - 2
    g = G.path_graph(3, np.array([2**31 - 1, 2**31 - 1], dtype=np.uint32))
    got, _ = gpu_solve(g, 2**31, [0])
    assert got[0].tolist() == [0, 2**31 - 1, 2**32 - 2]


def test_overflow_is_reported():
    g = G.path_graph(3, np.array([2**31, 2**31], dtype=np.uint32))
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 2**31)
    try:
        with pytest.raises(sssp.SsspError) as e:
            solver.solve([0])
        assert e.value.status == sssp.SSSP_ERR_OVERFLOW
        # an overflowing detour beside a representable path is fine
    finally:
        solver.close()
    g = G.csr_from_edges(3, np.array([0, 0, 1]), np.array([1, 2, 2]),
                         np.array([4_000_000_000, 5, 1_000_000_000], dtype=np.uint32))
    got, _ = gpu_solve(g, 10, [0])
    assert got[0].tolist() == [0, 4_000_000_000, 5]
    g = G.path_graph(3, np.array([3e38, 3e38], dtype=np.float32))
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 1e37)
    try:
        with pytest.raises(sssp.SsspError) as e:
            solver.solve([0])
        assert e.value.status == sssp.SSSP_ERR_OVERFLOW
    finally:
        solver.close()


def _create_status(row_ptr, col, w, delta):
    try:
        h = sssp.sssp_create(torch.from_numpy(row_ptr).cuda(), torch.from_numpy(col).cuda(),
                             torch.from_numpy(w).cuda(), delta)
    except sssp.SsspError as e:
        return e.status
    sssp.sssp_destroy(h)
    return sssp.SSSP_OK


def test_invalid_inputs_rejected():
    rp = np.array([0, 2, 3, 3], dtype=np.int64)
    col = np.array([1, 2, 0], dtype=np.int32)
    ok_w = np.array([1, 2, 3], dtype=np.int32)
    assert _create_status(rp, col, ok_w, 2) == sssp.SSSP_OK
    assert _create_status(rp, col, np.array([1, 0, 3], dtype=np.int32), 2) == sssp.SSSP_ERR_INVALID_WEIGHT
    for bad in (0.0, -1.0, np.nan, np.inf, -0.0):
        w = np.array([1.0, bad, 2.0], dtype=np.float32)
        assert _create_status(rp, col, w, 2.0) == sssp.SSSP_ERR_INVALID_WEIGHT, bad
    assert _create_status(rp, np.array([1, 3, 0], dtype=np.int32), ok_w, 2) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert _create_status(rp, np.array([1, -1, 0], dtype=np.int32), ok_w, 2) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert _create_status(np.array([0, 2, 1, 3], dtype=np.int64), col, ok_w, 2) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert _create_status(np.array([1, 2, 3, 3], dtype=np.int64), col, ok_w, 2) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert _create_status(np.array([0, 2, 3, 2], dtype=np.int64), col, ok_w, 2) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert _create_status(rp, col, ok_w, 2.5) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert _create_status(rp, col, ok_w, 0) == sssp.SSSP_ERR_INVALID_ARGUMENT
    # fp32: bucket indices of every possible distance (total weight times the
    # rounding factor, over delta) must fit 32 bits
    assert _create_status(rp, col, np.array([1e20, 1.0, 1.0], dtype=np.float32), 1e-3) == sssp.SSSP_ERR_UNSUPPORTED
    assert _create_status(rp, col, np.array([3e9, 2e9, 1.0], dtype=np.float32), 1.0) == sssp.SSSP_ERR_UNSUPPORTED
    assert _create_status(rp, col, np.array([1e9, 2e9, 1.0], dtype=np.float32), 1.0) == sssp.SSSP_OK
    g = G.workload("er_n1024_m8192")
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 32)
    try:
        for bad_src in ([-1], [1024], [0, 5000]):
            with pytest.raises(sssp.SsspError) as e:
                solver.solve(bad_src)
            assert e.value.status == sssp.SSSP_ERR_INVALID_ARGUMENT
        got = solver.solve_numpy([3])  # the handle stays usable after errors
        assert_exact(g, got[0], 3)
    finally:
        solver.close()


def test_fp32_bucket_indices_above_2_29():
    """Bucket indices up to about 3e9 (exact floor(t / delta) by a fused multiply-add sign test)."""
    g = G.path_graph(5, np.array([1e9, 1e9, 3.0, 1e9], dtype=np.float32))
    for delta in (1.0, 3.0, 0.75):
        if 3.0e9 * 1.0000001 / delta >= 2**32 - 256:
            continue
        got, _ = gpu_solve(g, delta, [0])
        assert_exact(g, got[0], 0, f"delta={delta}")


def test_long_inline_run_with_short_wait_limit():
    """A path of 300k vertices at delta 1: every bucket holds one vertex, so the whole solve runs
    as steps of the leader workgroup alone inside a single device-wide barrier, while every other
    workgroup waits in it. With a 100 ms wait limit, the leader's heartbeat (one per step) is what
    keeps the waits from aborting the solve; distances are the prefix sums."""
    n = 300_000
    g = G.path_graph(n, np.ones(n - 1, dtype=np.uint32))
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 1)
    try:
        solver.set_tuning(wait_limit_ms=100)
        assert sssp.sssp_get_tuning(solver.handle)["wait_limit_ms"] == 100
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        got = solver.solve_numpy([0])[0]
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = solver.stats()
    finally:
        solver.close()
    print(f"[parity] path n={n} delta=1: {ms:.1f} ms, {st['barriers']} barriers, {st['buckets']} buckets", flush=True)
    assert np.array_equal(got, np.arange(n, dtype=np.uint32))
    assert st["buckets"] == n
    assert ms > 200.0, "the solve ended before the wait limit could matter"


@pytest.mark.parametrize("tile", [{"hub_edges": 256}, {"hub_edges": 65536}, {"chunk_entries": 32},
                                  {"chunk_entries": 128, "inline_entries": 64},
                                  {"inline_entries": 1, "inline_edges": 1},
                                  {"hub_edges": 512, "chunk_entries": 64, "inline_entries": 512,
                                   "inline_edges": 65536, "workgroups_per_cu": 1}])
def test_tile_schedules_exact(tile):
    """Every tile schedule the autotuner may pick (hub threshold, chunk size, the limits of the
    steps one workgroup runs alone) gives the oracle's distances, u32 and fp32."""
    g = G.rmat_graph(14, 16, cfg=2)
    srcs = G.sources_with_outedges(g, 3, cfg=2)
    got, _ = gpu_solve(g, 32, srcs, tuning=tile)
    for r, s in enumerate(srcs):
        assert_exact(g, got[r], s, f"tile {tile}")
    gf = G.rmat_graph(13, 16, cfg=41, weights="f32_loguniform", wlo=1e-2, whi=1e2)
    sf = G.sources_with_outedges(gf, 2, cfg=41)
    got, _ = gpu_solve(gf, 0.5, sf, tuning={**tile, "concurrent_sources": 2})
    for r, s in enumerate(sf):
        assert_exact(gf, got[r], s, f"f32 tile {tile}")


def test_tuning_fields_resolved_and_checked():
    g = G.workload("er_n1024_m8192")
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 32)
    try:
        t = sssp.sssp_get_tuning(solver.handle)
        assert t["hub_edges"] == 1024 and t["inline_edges"] == 4096 and t["wait_limit_ms"] == 30000
        assert t["chunk_entries"] in (256, 512) and t["inline_entries"] == t["chunk_entries"]
        assert t["concurrent_sources"] == 1 and t["workgroups_per_cu"] == 2
        assert t["leader_chain"] == 2  # 8 edges per vertex: one light step at a time by default
        for bad in ({"hub_edges": 100}, {"hub_edges": 3000}, {"chunk_entries": 1024}, {"chunk_entries": 48},
                    {"inline_entries": 513}, {"wait_limit_ms": -1}, {"leader_chain": 3}, {"leader_chain": -1}):
            with pytest.raises(sssp.SsspError) as e:
                solver.set_tuning(**bad)
            assert e.value.status == sssp.SSSP_ERR_INVALID_ARGUMENT, bad
        solver.set_tuning(hub_edges=4096, chunk_entries=64, inline_entries=100)
        t = sssp.sssp_get_tuning(solver.handle)
        assert (t["hub_edges"], t["chunk_entries"], t["inline_entries"]) == (4096, 64, 100)
        assert_exact(g, solver.solve_numpy([9])[0], 9)
    finally:
        solver.close()


@pytest.mark.parametrize("chain", [1, 2])
def test_leader_chain_exact(chain):
    """The leader's chained light steps (leader_chain 1: the re-inserted vertices stay in LDS and the
    bucket's next light phase starts at once) and one light step at a time (2), each forced on every
    graph class: R-MAT u32, fp32 log-uniform (repeated rounds), fp64, ER u32 with small inline limits,
    a grid, and concurrent sources; all equal the oracle's distances."""
    cases = [
        (G.rmat_graph(13, 16, cfg=61), 16.0, {}),
        (G.rmat_graph(12, 16, cfg=62, weights="f32_loguniform", wlo=1e-2, whi=1e2), 0.37, {}),
        (G.rmat_graph(12, 16, cfg=63, weights="f64", wlo=0.1, whi=10.0), 1.0, {}),
        (G.er_graph(3000, 12000, cfg=64, wlo=1, whi=100), 40.0, {"inline_entries": 16, "inline_edges": 64}),
        (G.grid_graph(80, 80, cfg=65), 400.0, {}),
        (G.grid_graph(48, 48, cfg=66), 100.0, {"concurrent_sources": 4}),
    ]
    for g, delta, extra in cases:
        srcs = G.sources_with_outedges(g, 3, cfg=60)
        got, st = gpu_solve(g, delta, srcs, tuning={"leader_chain": chain, **extra})
        for r, s in enumerate(srcs):
            assert_exact(g, got[r], s, f"{g.name} chain={chain} {extra}")
        assert st["sources"] == len(srcs)


def test_leader_chain_default_by_degree():
    """Chained light steps are the default on graphs of at most 6 edges per vertex (a grid: 4),
    one light step at a time on denser ones (R-MAT edge factor 16)."""
    for g, want in ((G.grid_graph(32, 32, cfg=67), 1), (G.rmat_graph(10, 16, cfg=67), 2)):
        solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 64)
        try:
            assert sssp.sssp_get_tuning(solver.handle)["leader_chain"] == want, g.name
            solver.set_tuning(leader_chain=3 - want)
            assert sssp.sssp_get_tuning(solver.handle)["leader_chain"] == 3 - want
        finally:
            solver.close()


def test_tuning_variants_agree():
    g = G.rmat_graph(12, 16, cfg=2)
    s = int(G.sources_with_outedges(g, 1, cfg=3)[0])
    for wpc in (1, 2, 4):
        got, _ = gpu_solve(g, 16, [s], tuning={"workgroups_per_cu": wpc})
        assert_exact(g, got[0], s, f"wg/cu={wpc}")


@pytest.fixture(scope="module")
def rmat_s22():
    return G.workload("rmat_s22_u32")


def test_rmat_s22_bench_configuration(rmat_s22):
    """The benchmark's launch: R-MAT scale 22, 64 sources in one call, delta 64. Rows 0, 1 and 63
    are compared with the oracle's Dijkstra vertex by vertex; all 64 rows are checked by the
    optimality certificate (a proof of exactness)."""
    print("[parity] rmat s22 delta=64, 64 sources", flush=True)
    g = rmat_s22
    srcs = G.sources_with_outedges(g, 64, cfg=2)
    got, st = gpu_solve(g, 64, srcs)
    assert st["sources"] == 64
    for r in (0, 1, 63):
        assert_exact(g, got[r], srcs[r], "rmat s22 delta=64")
    certify_rows(g, srcs, got, "rmat s22 delta=64")


@pytest.mark.parametrize("delta", [8, 16, 32, 128])
def test_rmat_s22_swept_deltas(rmat_s22, delta):
    """Every other delta of the benchmark's sweep: two of the 64 sources per delta, each compared
    with Dijkstra vertex by vertex (a different pair of rows for every delta)."""
    print(f"[parity] rmat s22 delta={delta}", flush=True)
    g = rmat_s22
    all_srcs = G.sources_with_outedges(g, 64, cfg=2)
    pick = {8: (63, 5), 16: (10, 40), 32: (20, 50), 128: (30, 60)}[delta]
    srcs = all_srcs[list(pick)]
    got, _ = gpu_solve(g, delta, srcs)
    for r, s in enumerate(srcs):
        assert_exact(g, got[r], s, f"rmat s22 delta={delta}")


@pytest.fixture(scope="module")
def grid4096():
    return G.workload("grid4096_u32")


@pytest.mark.parametrize("delta", [50, 100, 400])
def test_grid_4096_many_buckets(grid4096, delta):
    """The high-diameter grid at each delta of the benchmark (about 4.7k to 37k buckets with small
    frontiers, corner source): certified, and compared with Dijkstra vertex by vertex."""
    print(f"[parity] grid 4096 delta={delta}", flush=True)
    g = grid4096
    got, st = gpu_solve(g, delta, [0])
    assert oracle.certify(g, 0, got[0]) == oracle.CERT_OK
    assert_exact(g, got[0], 0, f"grid4096 delta={delta}")
    assert st["buckets"] >= len(np.unique(got[0] // delta))


# ---------------------------------------------------------------- fp64 weights (the paper's GrB_FP64)

@pytest.mark.parametrize("delta", [0.25, 1.0, 7.5])
def test_fp64_rmat_exact(delta):
    """fp64 weights uniform in [0.1, 10): distances equal Dijkstra's in binary64, bit for bit."""
    g = G.rmat_graph(13, 16, cfg=91, weights="f64", wlo=0.1, whi=10.0)
    srcs = G.sources_with_outedges(g, 3, cfg=91)
    got, st = gpu_solve(g, delta, srcs)
    assert got.dtype == np.float64
    for r, s in enumerate(srcs):
        assert_exact(g, got[r], s, f"f64 delta={delta}")
    assert st["sources"] == len(srcs)


def test_fp64_groups_multi_and_weights():
    g = G.er_graph(4000, 32000, cfg=92, weights="f64", wlo=1e-3, whi=1.0)
    srcs = G.sources_with_outedges(g, 12, cfg=92)
    got, _ = gpu_solve(g, 2.0 ** -5, srcs, tuning={"concurrent_sources": 8})
    for r, s in enumerate(srcs):
        assert_exact(g, got[r], s, "f64 groups")
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 0.1)
    try:
        d = solver.solve_multi(srcs[:4]).cpu().numpy()
        want = np.stack([oracle.dijkstra(g, int(s))[0] for s in srcs[:4]]).min(axis=0)
        assert np.array_equal(_bits(d), _bits(want))
        w2 = (g.w * 3.0 + 0.5).astype(np.float64)  # new weights: larger spread, same structure
        solver.set_weights(w2)
        g2 = G.Graph(n=g.n, row_ptr=g.row_ptr, col=g.col, w=w2)
        d2 = solver.solve_numpy(srcs[:2])
        for r, s in enumerate(srcs[:2]):
            assert_exact(g2, d2[r], s, "f64 set_weights")
        with pytest.raises(sssp.SsspError) as e:  # the adjoint is fp32 only
            solver.backward(srcs[:1], torch.from_numpy(d2[:1]).cuda(), torch.ones((1, g.n), device="cuda"))
        assert e.value.status == sssp.SSSP_ERR_UNSUPPORTED
    finally:
        solver.close()


def test_fp64_invalid_weights_and_overflow():
    rp = np.array([0, 2, 3, 3], dtype=np.int64)
    col = np.array([1, 2, 0], dtype=np.int32)
    for bad in (0.0, -1.0, np.nan, np.inf, -0.0, -np.inf):
        w = np.array([1.0, bad, 2.0], dtype=np.float64)
        assert _create_status(rp, col, w, 2.0) == sssp.SSSP_ERR_INVALID_WEIGHT, bad
    assert _create_status(rp, col, np.array([1.0, 5e-324, 2.0]), 1.0) == sssp.SSSP_OK  # subnormal is positive
    assert _create_status(rp, col, np.array([1e300, 1.0, 1.0]), 1e-300) == sssp.SSSP_ERR_UNSUPPORTED
    # a total weight beyond the fp64 range fails the bucket-range bound, so no fp64 path sum can overflow
    assert _create_status(rp, col, np.array([1.7e308, 1.7e308, 1.0]), 1e300) == sssp.SSSP_ERR_UNSUPPORTED
    g = G.path_graph(3, np.array([1.7e308, 1.0], dtype=np.float64))
    got, _ = gpu_solve(g, 1e300, [0])
    assert got[0].tolist() == [0.0, 1.7e308, 1.7e308]
