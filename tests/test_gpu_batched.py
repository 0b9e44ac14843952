"""Concurrent sources (several workgroup groups in one launch), the enqueue-only
entry point with device-resident sources, and its capture into a HIP graph,
against the CPU oracle (Dijkstra rows bit-exact, or the O(m) certificate)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1911_06895_amd import graphs as G  # noqa: E402
from paper_1911_06895_amd import sssp  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU-only hosts
    pytest.skip("no GPU", allow_module_level=True)


def as_host(dist, wdtype):
    d = dist.cpu().numpy()
    return d.view(np.uint32) if wdtype == np.uint32 else d


def same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint32), np.asarray(b).view(np.uint32))


def check_rows(g, srcs, rows, exact_rows=4):
    """The first rows against Dijkstra bit for bit, every row by the certificate."""
    for r, s in enumerate(srcs):
        if r < exact_rows:
            want, rc = oracle.dijkstra(g, int(s))
            assert rc == oracle.OK
            assert same_bits(rows[r], want), f"row {r} (source {s}) differs from Dijkstra"
        else:
            assert oracle.certify(g, int(s), rows[r]) == oracle.CERT_OK, f"row {r} (source {s}) not certified"


@pytest.mark.parametrize("groups", [2, 8, 32, 256])
@pytest.mark.parametrize("kind", ["u32", "f32_loguniform"])
def test_concurrent_groups_match_oracle(groups, kind):
    print(f"[batched] groups={groups} kind={kind}", flush=True)
    if kind == "u32":
        g, delta = G.rmat_graph(14, 16, cfg=61, weights="u32", wlo=1, whi=255), 32
    else:
        g, delta = G.rmat_graph(14, 16, cfg=62, weights="f32_loguniform", wlo=1e-2, whi=1e2), 2.0 ** -5
    srcs = G.sources_with_outedges(g, 3 * groups // 2 + 5, cfg=61)  # more sources than groups, not a multiple
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, delta)
    try:
        solver.set_tuning(concurrent_sources=groups)
        rows = solver.solve_numpy(srcs)
        st = solver.stats()
        assert st["sources"] == len(srcs)
        check_rows(g, srcs, rows, exact_rows=6)
        solver.set_tuning(concurrent_sources=1)  # one group: the same rows, bit for bit
        assert np.array_equal(rows.view(np.uint32), solver.solve_numpy(srcs).view(np.uint32))
    finally:
        solver.close()


@pytest.mark.parametrize("groups,wpc,kind", [(1, 0, "u32"), (2, 0, "u32"), (1, 1, "u32"), (2, 0, "f32_loguniform"),
                                             (16, 0, "f32_loguniform")])
def test_reused_distance_buffers(groups, wpc, kind):
    """Hundreds of rows per group in one launch: each of a group's two distance
    buffers serves every other row, so the cached copies an earlier row leaves
    must never feed the next row's prefilter. Every row is certified, over
    three launches (wpc 1: the 1024-thread workgroup configuration)."""
    print(f"[batched] reused buffers groups={groups} workgroups_per_cu={wpc} kind={kind}", flush=True)
    if kind == "u32":
        g, delta = G.rmat_graph(14, 16, cfg=61, weights="u32", wlo=1, whi=255), 32
    else:
        g, delta = G.rmat_graph(14, 16, cfg=62, weights="f32_loguniform", wlo=1e-2, whi=1e2), 2.0 ** -5
    srcs = G.sources_with_outedges(g, 401, cfg=64)
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, delta)
    try:
        solver.set_tuning(concurrent_sources=groups, workgroups_per_cu=wpc)
        for launch in range(3):
            rows = solver.solve_numpy(srcs)
            check_rows(g, srcs, rows, exact_rows=2 if launch == 0 else 0)
    finally:
        solver.close()


def test_c4a_configuration():
    """R-MAT scale 18, fp32 log-uniform weights in [1e-2, 1e2], 256 sources, 8 groups."""
    print("[batched] C4a rmat_s18_f32log k=256 groups=8", flush=True)
    g = G.workload("rmat_s18_f32log")
    srcs = G.sources_with_outedges(g, 256, cfg=41)
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 2.0 ** -5)
    try:
        solver.set_tuning(concurrent_sources=8)
        rows = solver.solve_numpy(srcs)
        assert solver.stats()["sources"] == 256
    finally:
        solver.close()
    check_rows(g, srcs, rows, exact_rows=3)


def test_async_device_sources_and_status():
    g = G.er_graph(5000, 40000, cfg=63, weights="u32", wlo=1, whi=100)
    srcs = np.array([0, 17, 4999, 2500, 3], dtype=np.int32)
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 16)
    try:
        solver.set_tuning(concurrent_sources=4)
        src_dev = torch.from_numpy(srcs).cuda()
        dist = torch.empty((len(srcs), g.n), dtype=torch.int32, device="cuda")
        sssp.sssp_solve_async(solver.handle, src_dev, dist)
        sssp.sssp_solve_status(solver.handle)
        check_rows(g, srcs, as_host(dist, np.uint32), exact_rows=len(srcs))
        # a source outside [0, n): its row is all-unreachable, the others are correct, the status says so
        bad = torch.tensor([5, g.n, 9], dtype=torch.int32, device="cuda")
        dist2 = torch.empty((3, g.n), dtype=torch.int32, device="cuda")
        sssp.sssp_solve_async(solver.handle, bad, dist2)
        with pytest.raises(sssp.SsspError) as e:
            sssp.sssp_solve_status(solver.handle)
        assert e.value.status == sssp.SSSP_ERR_INVALID_ARGUMENT
        d2 = as_host(dist2, np.uint32)
        assert np.all(d2[1] == np.uint32(0xFFFFFFFF))
        check_rows(g, [5, 9], d2[[0, 2]], exact_rows=2)
        # the handle stays usable
        sssp.sssp_solve_async(solver.handle, src_dev, dist)
        sssp.sssp_solve_status(solver.handle)
    finally:
        solver.close()


def test_status_without_enqueue_and_bad_tuning():
    g = G.er_graph(300, 2000, cfg=64, weights="u32", wlo=1, whi=9)
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 4)
    try:
        with pytest.raises(sssp.SsspError) as e:
            sssp.sssp_solve_status(solver.handle)
        assert e.value.status == sssp.SSSP_ERR_NO_FORWARD
        for bad in (3, 512):  # not a divisor of the workgroup count / above the limit
            with pytest.raises(sssp.SsspError) as e:
                solver.set_tuning(concurrent_sources=bad)
            assert e.value.status == sssp.SSSP_ERR_UNSUPPORTED
        with pytest.raises(sssp.SsspError) as e:
            solver.set_tuning(concurrent_sources=-1)
        assert e.value.status == sssp.SSSP_ERR_INVALID_ARGUMENT
        rows = solver.solve_numpy([0, 1])  # the failed calls left the handle as it was
        check_rows(g, [0, 1], rows, exact_rows=2)
    finally:
        solver.close()


@pytest.mark.parametrize("groups", [1, 8])
def test_graph_capture_replays(groups):
    """sssp_solve_async recorded into a HIP graph by stream capture; every replay (with new
    sources written into the captured buffer, and eager work in between) equals an eager solve."""
    print(f"[batched] graph capture groups={groups}", flush=True)
    g = G.rmat_graph(13, 16, cfg=65, weights="f32_loguniform", wlo=1e-2, whi=1e2)
    cand = G.sources_with_outedges(g, 48, cfg=65)
    k = 16
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 2.0 ** -4)
    try:
        solver.set_tuning(concurrent_sources=groups)
        src_static = torch.from_numpy(cand[:k].astype(np.int32)).cuda()
        out_static = torch.empty((k, g.n), dtype=torch.float32, device="cuda")
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):  # warm up on the capture stream
            sssp.sssp_solve_async(solver.handle, src_static, out_static, stream)
        sssp.sssp_solve_status(solver.handle, stream)
        torch.cuda.current_stream().wait_stream(stream)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            sssp.sssp_solve_async(solver.handle, src_static, out_static, stream)
        for rep in range(3):
            batch = cand[rep * k:(rep + 1) * k].astype(np.int32)
            src_static.copy_(torch.from_numpy(batch))
            graph.replay()
            torch.cuda.synchronize()
            sssp.sssp_solve_status(solver.handle, torch.cuda.current_stream())
            got = out_static.cpu().numpy()
            eager = solver.solve_numpy(batch)  # eager work between replays
            assert same_bits(got, eager), f"replay {rep} differs from the eager solve"
            check_rows(g, batch, got, exact_rows=2)
        del graph
    finally:
        torch.cuda.synchronize()
        solver.close()


@pytest.mark.parametrize("kind", ["u32", "f32_unit"])
def test_multi_source_is_min_over_sources(kind):
    """sssp_solve_multi: d(v) = min over the sources of d_s(v) (repeated sources allowed)."""
    if kind == "u32":
        g, delta = G.rmat_graph(12, 8, cfg=66, weights="u32", wlo=1, whi=64), 16
    else:
        g, delta = G.rmat_graph(12, 8, cfg=67, weights="f32_unit"), 2.0 ** -4
    srcs = np.concatenate([G.sources_with_outedges(g, 7, cfg=66), [0, 0]]).astype(np.int32)
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, delta)
    try:
        got = solver.solve_multi(srcs).cpu().numpy()
        assert solver.stats()["sources"] == 1
    finally:
        solver.close()
    rows = np.stack([oracle.dijkstra(g, int(s))[0] for s in srcs])
    want = rows.min(axis=0)
    assert same_bits(got.view(want.dtype), want)


def _check_blocks(graphs, offs, dist, exact_blocks):
    """Each block's slice of the union's distances against its own graph's oracle."""
    for i, gi in enumerate(graphs):
        seg = dist[offs[i]:offs[i + 1]]
        if i in exact_blocks:
            want, rc = oracle.dijkstra(gi, 0)
            assert rc == oracle.OK and same_bits(seg, want), f"block {i} (n={gi.n}) differs from Dijkstra"
        else:
            assert oracle.certify(gi, 0, seg) == oracle.CERT_OK, f"block {i} (n={gi.n}) not certified"


def test_ragged_batch_small():
    """64 ER graphs (n log-uniform in [1e3, 1e4], degree 8, fp32 weights in (0, 1]) as one
    block-diagonal graph, one source per block, one multi-source solve."""
    graphs = G.ragged_er_batch(64, cfg=68, nlo=1_000, nhi=10_000)
    u, offs = G.block_union(graphs)
    solver = sssp.DeltaStepping(u.row_ptr, u.col, u.w, 0.125)
    try:
        dist = solver.solve_multi(offs[:-1].astype(np.int32)).cpu().numpy()
    finally:
        solver.close()
    _check_blocks(graphs, offs, dist, exact_blocks=set(range(64)))


def test_c4b_configuration():
    """512 ER graphs, n log-uniform in [1e3, 1e5], degree 8, fp32 weights in (0, 1]: the union
    solved from the first vertex of every block at once, captured in a graph and replayed."""
    print("[batched] C4b ragged_er512", flush=True)
    graphs = G.ragged_er_batch(512, cfg=42)
    u, offs = G.block_union(graphs)
    solver = sssp.DeltaStepping(u.row_ptr, u.col, u.w, 0.125)
    try:
        src = torch.from_numpy(offs[:-1].astype(np.int32)).cuda()
        dist = torch.empty(u.n, dtype=torch.float32, device="cuda")
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            sssp.sssp_solve_multi_async(solver.handle, src, dist, stream)
        sssp.sssp_solve_status(solver.handle, stream)
        first = dist.cpu().numpy()
        torch.cuda.current_stream().wait_stream(stream)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            sssp.sssp_solve_multi_async(solver.handle, src, dist, stream)
        for _ in range(2):
            dist.fill_(0.0)
            graph.replay()
            torch.cuda.synchronize()
            sssp.sssp_solve_status(solver.handle, torch.cuda.current_stream())
            assert same_bits(dist.cpu().numpy(), first)
        del graph
    finally:
        torch.cuda.synchronize()
        solver.close()
    _check_blocks(graphs, offs, first, exact_blocks=set(range(0, 512, 37)))


def test_bfs_mode_unit_weights():
    """Undirected unit weights with delta = 1 (the paper's own experimental setting):
    distances are BFS hop counts, every edge is light, one light phase per bucket."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path

    g = G.symmetrize(G.rmat_graph(14, 8, cfg=69, weights="u32", wlo=1, whi=1))
    src = int(G.sources_with_outedges(g, 1, cfg=69)[0])
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 1)
    try:
        got = solver.solve_numpy([src])[0]
        st = solver.stats()
    finally:
        solver.close()
    orc, rc = oracle.dijkstra(g, src)
    assert rc == oracle.OK and np.array_equal(got, orc), "BFS mode differs from the oracle's Dijkstra"
    a = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    hops = shortest_path(a, method="D", unweighted=True, indices=src)
    want = np.where(np.isfinite(hops), hops, 2.0 ** 32 - 1).astype(np.uint32)
    assert np.array_equal(got, want)
    assert st["heavy_phases"] == 0 and st["heavy_edges"] == 0
    assert st["light_phases"] == st["buckets"]  # the level of bucket i only reaches bucket i + 1
    assert st["buckets"] == int(hops[np.isfinite(hops)].max()) + 1


def test_autotune_returns_a_correct_tuned_handle():
    g = G.rmat_graph(13, 16, cfg=70, weights="f32_loguniform", wlo=1e-2, whi=1e2)
    srcs = G.sources_with_outedges(g, 32, cfg=70)
    rp, ci = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
    wt = torch.from_numpy(g.w).cuda()
    scratch = torch.empty((len(srcs), g.n), dtype=torch.float32, device="cuda")
    h, res = sssp.sssp_autotune(rp, ci, wt, srcs, scratch)
    try:
        assert res["trials"] >= 2 and res["ms"] > 0
        tiles = res["tuning"]
        assert tiles == sssp.sssp_get_tuning(h)
        assert tiles["hub_edges"] in (512, 1024, 2048, 4096) and tiles["chunk_entries"] in (64, 128, 256, 512)
        assert tiles["concurrent_sources"] == res["concurrent_sources"]
        mean = float(g.w.astype(np.float64).mean())
        assert mean / 64 <= res["delta"] <= mean * 8 and np.log2(res["delta"]).is_integer()
        assert res["concurrent_sources"] in (1, 8, 16, 32)
        dist = torch.empty((4, g.n), dtype=torch.float32, device="cuda")
        sssp.sssp_solve(h, srcs[:4], dist)
        check_rows(g, srcs[:4], dist.cpu().numpy(), exact_rows=4)
    finally:
        sssp.sssp_destroy(h)
    # nearest-source mode with explicit candidates
    h, res = sssp.sssp_autotune(rp, ci, wt, srcs[:3], scratch[0], multi=True, deltas=[0.5, 2.0])
    try:
        # two (delta, group) trials, then the tile search on the faster one
        assert res["delta"] in (0.5, 2.0) and res["concurrent_sources"] == 1 and res["trials"] > 2
        d = torch.empty(g.n, dtype=torch.float32, device="cuda")
        sssp.sssp_solve_multi(h, srcs[:3], d)
        want = np.stack([oracle.dijkstra(g, int(s))[0] for s in srcs[:3]]).min(axis=0)
        assert same_bits(d.cpu().numpy(), want)
    finally:
        sssp.sssp_destroy(h)


def test_autotuned_tiles_exact_rmat_and_ragged():
    """Handles the autotuner returns (delta, groups and the tile schedule chosen by timing) are
    oracle-exact: R-MAT scale 14 with u32 weights, and the ragged batch in nearest-source mode."""
    print("[batched] autotuned tiles: rmat s14 u32 and a ragged batch", flush=True)
    g = G.rmat_graph(14, 16, cfg=2)
    srcs = G.sources_with_outedges(g, 24, cfg=2)
    rp, ci = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
    wt = torch.from_numpy(g.w.view(np.int32)).cuda()
    scratch = torch.empty((len(srcs), g.n), dtype=torch.int32, device="cuda")
    h, res = sssp.sssp_autotune(rp, ci, wt, srcs, scratch)
    try:
        print(f"[batched] rmat s14 tuned: delta {res['delta']}, {res['tuning']}", flush=True)
        dist = torch.empty((len(srcs), g.n), dtype=torch.int32, device="cuda")
        sssp.sssp_solve(h, srcs, dist)
        check_rows(g, srcs, as_host(dist, np.uint32), exact_rows=len(srcs))
    finally:
        sssp.sssp_destroy(h)
    graphs = G.ragged_er_batch(96, cfg=68, nlo=1_000, nhi=20_000)
    u, offs = G.block_union(graphs)
    starts = offs[:-1].astype(np.int32)
    rp, ci, wt = (torch.from_numpy(a).cuda() for a in (u.row_ptr, u.col, u.w))
    d = torch.empty(u.n, dtype=torch.float32, device="cuda")
    h, res = sssp.sssp_autotune(rp, ci, wt, starts, d, multi=True)
    try:
        print(f"[batched] ragged tuned: delta {res['delta']}, {res['tuning']}", flush=True)
        d.fill_(0.0)
        sssp.sssp_solve_multi(h, starts, d)
        _check_blocks(graphs, offs, d.cpu().numpy(), exact_blocks=set(range(96)))
    finally:
        sssp.sssp_destroy(h)
