"""The seeded input generators (no GPU): each workload recipe holds the
structure and value ranges it claims, and the same seed gives the same graph."""
import math

import numpy as np

from paper_1911_06895_amd import graphs as G


def pairs(g):
    return g.edge_src().astype(np.int64), g.col.astype(np.int64)


def assert_simple(g):
    g.check()
    s, d = pairs(g)
    assert np.all(s != d), "self-loop"
    key = s * g.n + d
    assert np.all(np.diff(key) > 0), "rows sorted by destination, no parallel edges"


def test_er_correctness_gate_graph():
    g = G.workload("er_n1024_m8192")
    assert (g.n, g.m) == (1024, 8192)
    assert_simple(g)
    assert g.w.dtype == np.uint32 and g.w.min() >= 1 and g.w.max() <= 100


def test_rmat_structure_and_weights():
    g = G.rmat_graph(12, 16, cfg=2, weights="u32", wlo=1, whi=255)
    assert g.n == 4096 and 0 < g.m <= 16 * 4096
    assert_simple(g)
    assert g.w.dtype == np.uint32 and g.w.min() >= 1 and g.w.max() <= 255
    deg = g.outdeg()
    assert deg.max() >= 20 * deg.mean(), "R-MAT degrees are heavily skewed"
    assert int(np.argmax(deg)) != 0, "ids are permuted: the hub is not vertex 0"


def test_rmat_quadrant_probabilities():
    """Every bit level of (src, dst): quadrant (0,0) with a, (0,1) with b, (1,0) with c,
    (1,1) with d (b != c, so a swap of source and destination bits shows)."""
    src, dst = G.rmat_pairs(G.rng_for(7, 1), 10, 200_000, 0.50, 0.30, 0.15)
    for level in (9, 4, 0):
        bit = 1 << level
        sb, db = (src & bit) != 0, (dst & bit) != 0
        freq = [np.mean(~sb & ~db), np.mean(~sb & db), np.mean(sb & ~db), np.mean(sb & db)]
        for got, want in zip(freq, (0.50, 0.30, 0.15, 0.05)):
            assert abs(got - want) < 0.005, (level, freq, "quadrant frequencies")


def test_grid_is_four_neighbour():
    rows, cols = 5, 7
    g = G.grid_graph(rows, cols, cfg=3, weights="u32", wlo=1, whi=1000)
    assert g.n == rows * cols and g.m == 2 * (2 * rows * cols - rows - cols)
    assert_simple(g)
    s, d = pairs(g)
    dr, dc = np.abs(s // cols - d // cols), np.abs(s % cols - d % cols)
    assert np.all(dr + dc == 1), "edges join 4-neighbours"
    deg = g.outdeg().reshape(rows, cols)
    assert deg[0, 0] == 2 and deg[0, 3] == 3 and deg[2, 3] == 4
    assert g.w.min() >= 1 and g.w.max() <= 1000


def test_weight_distributions():
    rng = G.rng_for(5, 2)
    lw = G.weights_loguniform_f32(rng, 200_000, 1e-2, 1e2)
    assert lw.dtype == np.float32 and lw.min() >= np.float32(1e-2) and lw.max() <= np.float32(1e2)
    assert abs(float(np.mean(np.log(lw.astype(np.float64))))) < 0.02, "log-uniform: mean log near 0"
    uw = G.weights_unit_interval_f32(rng, 100_000)
    k = uw.astype(np.float64) * (1 << 24)
    assert uw.min() > 0 and uw.max() <= 1 and np.all(k == np.round(k)), "(k+1)/2^24 in (0, 1]"
    ow = G.weights_one_two_f32(rng, 100_000)
    k = (ow.astype(np.float64) - 1.0) * (1 << 23)
    assert ow.min() >= 1 and ow.max() < 2 and np.all(k == np.round(k)), "1 + k/2^23 in [1, 2)"


def test_ragged_batch_and_block_union():
    graphs = G.ragged_er_batch(8, cfg=42)
    for g in graphs:
        assert 1_000 <= g.n <= 100_000 and g.m == 8 * g.n
        assert_simple(g)
        assert g.w.dtype == np.float32 and g.w.min() > 0 and g.w.max() <= 1
    u, offs = G.block_union(graphs)
    assert u.n == sum(g.n for g in graphs) and u.m == sum(g.m for g in graphs)
    u.check()
    assert list(offs) == [0] + list(np.cumsum([g.n for g in graphs]))
    s, d = pairs(u)
    block = np.searchsorted(offs, s, side="right") - 1
    assert np.all((d >= offs[block]) & (d < offs[block + 1])), "block-diagonal: no edge leaves its graph"
    g3 = graphs[3]
    s3, d3 = pairs(g3)
    us, ud = s[u.row_ptr[offs[3]]:u.row_ptr[offs[4]]], d[u.row_ptr[offs[3]]:u.row_ptr[offs[4]]]
    assert np.array_equal(us - offs[3], s3) and np.array_equal(ud - offs[3], d3)


def test_sizes_are_log_uniform():
    sizes = np.array([g.n for g in G.ragged_er_batch(64, cfg=9, nlo=10, nhi=1000)], dtype=np.float64)
    mid = math.log(100)
    logs = np.log(sizes)
    assert logs.min() >= math.log(10) - 0.05 and logs.max() <= math.log(1000) + 0.05
    assert abs(np.mean(logs) - mid) < 0.35, "mean of log n near the middle of the range"


def test_sources_targets_and_determinism():
    g = G.rmat_graph(10, 16, cfg=4)
    srcs = G.sources_with_outedges(g, 64, cfg=2)
    assert srcs.size == 64 and np.unique(srcs).size == 64 and np.all(g.outdeg()[srcs] > 0)
    t, c = G.targets_and_coefs(g.n, 100, cfg=5)
    assert np.unique(t).size == 100 and t.min() >= 0 and t.max() < g.n and c.dtype == np.float32
    again = G.rmat_graph(10, 16, cfg=4)
    assert np.array_equal(g.row_ptr, again.row_ptr) and np.array_equal(g.col, again.col)
    assert np.array_equal(g.w, again.w)
    other = G.rmat_graph(10, 16, cfg=5)
    assert not (other.m == g.m and np.array_equal(other.col, g.col)), "another seed, another graph"
    assert np.array_equal(srcs, G.sources_with_outedges(g, 64, cfg=2))


def test_parallel_edges_keep_their_minimum_and_self_loops_go():
    src = np.array([0, 0, 2, 1, 0, 1])
    dst = np.array([1, 1, 2, 0, 2, 0])
    for w in (np.array([5, 3, 7, 9, 4, 8], dtype=np.uint32),  # packed-key path
              np.array([5, 3, 7, 9, 4, 8], dtype=np.float32)):  # sort path
        g = G.csr_from_edges(3, src, dst, w)
        assert_simple(g)
        s, d = pairs(g)
        assert list(zip(s.tolist(), d.tolist(), g.w.tolist())) == [(0, 1, 3), (0, 2, 4), (1, 0, 8)]
