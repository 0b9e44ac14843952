"""sssp_backward_noalloc (the adjoint with its working set in the library's static device array,
for callers that cannot allocate) against sssp_backward on the same handle, through the C ABI:
two calls in a row, the second on a smaller graph with fewer sources, each compared to the
1e-6 relative bar (integer subtree sizes bit for bit), plus its size limit and error paths."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from conftest import report  # noqa: E402
from paper_1911_06895_amd import graphs as G  # noqa: E402
from paper_1911_06895_amd import sssp  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU-only hosts
    pytest.skip("no GPU", allow_module_level=True)


def _both(g, delta, srcs, grad_rows, groups):
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, delta)
    try:
        solver.set_tuning(concurrent_sources=groups)
        dist = solver.solve(srcs)
        gd = torch.from_numpy(np.ascontiguousarray(grad_rows, dtype=np.float32)).cuda()
        ref = torch.empty(g.m, dtype=torch.float32, device="cuda")
        sssp.sssp_backward(solver.handle, srcs, dist, gd, ref)
        got = torch.full((g.m,), float("nan"), dtype=torch.float32, device="cuda")
        src_dev = torch.from_numpy(np.asarray(srcs, dtype=np.int32)).cuda()
        sssp.sssp_backward_noalloc(solver.handle, src_dev, dist, gd, got)
        return dist.cpu().numpy(), ref.cpu().numpy(), got.cpu().numpy()
    finally:
        solver.close()


def _close(got, ref, what):
    err = np.abs(got.astype(np.float64) - ref.astype(np.float64))
    nz = ref != 0
    rel = err[nz] / np.abs(ref[nz].astype(np.float64)) if nz.any() else np.zeros(1)
    report(f"[no-alloc] {what}: max abs diff {err.max():.3e}, max rel diff {rel.max():.3e}")
    assert np.all(err <= 1e-6 * np.abs(ref.astype(np.float64))), what


def test_noalloc_matches_backward_twice_second_smaller():
    print("[no-alloc] call 1: R-MAT scale 14, fp32 [1,2), 8 sources, 4 groups", flush=True)
    g1 = G.rmat_graph(14, 16, cfg=5, weights="f32_one_two")
    s1 = G.sources_with_outedges(g1, 8, cfg=5)
    t1, c1 = G.targets_and_coefs(g1.n, 512, cfg=5)
    r1 = np.zeros((len(s1), g1.n))
    r1[:, t1] = c1
    d1, ref1, got1 = _both(g1, 0.5, s1, r1, groups=4)
    for r, s in enumerate(s1[:2]):
        want, _ = oracle.dijkstra(g1, int(s))
        assert np.array_equal(d1[r].view(np.uint32), want.view(np.uint32))
    _close(got1, ref1, "call 1")
    print("[no-alloc] call 2: ER n=3000 m=24000, 3 sources, subtree sizes", flush=True)
    g2 = G.er_graph(3000, 24000, cfg=88, weights="f32_one_two")
    s2 = G.sources_with_outedges(g2, 3, cfg=88)
    solver = sssp.DeltaStepping(g2.row_ptr, g2.col, g2.w, 0.25)
    try:
        dist = solver.solve(s2)
        ones = torch.isfinite(dist).float()
        ref = torch.empty(g2.m, dtype=torch.float32, device="cuda")
        sssp.sssp_backward(solver.handle, s2, dist, ones, ref)
        got = torch.full((g2.m,), float("nan"), dtype=torch.float32, device="cuda")
        sssp.sssp_backward_noalloc(solver.handle, torch.from_numpy(s2.astype(np.int32)).cuda(), dist, ones, got)
        d2 = dist.cpu().numpy()
    finally:
        solver.close()
    assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy()), "integer subtree sizes differ"
    want = np.zeros(g2.m)
    for r, s in enumerate(s2):
        oracle.sp_gradient(g2, int(s), d2[r], np.isfinite(d2[r]).astype(np.float64), want)
    assert np.array_equal(got.cpu().numpy().astype(np.float64), want)


def test_noalloc_limits_and_errors():
    # one group of this graph does not fit the array (8 bytes per edge alone exceed it)
    r = G.rng_for(89, G.S_STRUCT)
    m = 9_000_000
    g = G.csr_from_edges(64, r.integers(0, 64, m), r.integers(0, 64, m),
                         (1.0 + r.random(m)).astype(np.float32), dedup=False)
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 1.0)
    try:
        dist = solver.solve([0])
        gd = torch.ones_like(dist)
        gw = torch.empty(g.m, dtype=torch.float32, device="cuda")
        with pytest.raises(sssp.SsspError) as e:
            sssp.sssp_backward_noalloc(solver.handle, torch.zeros(1, dtype=torch.int32, device="cuda"), dist, gd, gw)
        assert e.value.status == sssp.SSSP_ERR_UNSUPPORTED
        sssp.sssp_backward(solver.handle, [0], dist, gd, gw)  # the allocating entry point still works
    finally:
        solver.close()
    g = G.er_graph(500, 3000, cfg=90, weights="f32_one_two")
    solver = sssp.DeltaStepping(g.row_ptr, g.col, g.w, 0.5)
    try:
        gw = torch.empty(g.m, dtype=torch.float32, device="cuda")
        src = torch.tensor([0, 7], dtype=torch.int32, device="cuda")
        dist = torch.zeros((2, g.n), dtype=torch.float32, device="cuda")
        with pytest.raises(sssp.SsspError) as e:
            sssp.sssp_backward_noalloc(solver.handle, src, dist, torch.ones_like(dist), gw)
        assert e.value.status == sssp.SSSP_ERR_NO_FORWARD
        dist = solver.solve([0, 7])
        bad = torch.tensor([0, g.n], dtype=torch.int32, device="cuda")
        with pytest.raises(sssp.SsspError) as e:
            sssp.sssp_backward_noalloc(solver.handle, bad, dist, torch.ones_like(dist), gw)
        assert e.value.status == sssp.SSSP_ERR_INVALID_ARGUMENT
        sssp.sssp_backward_noalloc(solver.handle, src, dist, torch.isfinite(dist).float(), gw)
    finally:
        solver.close()
