"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each ``pin_*`` takes a loaded oracle build and returns a list of failure
messages (empty = pinned). The test module asserts each pin on the real build;
the planted-mistake test runs them all on deliberately broken builds and
requires that every planted mistake trips at least one pin.

Sources of truth used here (none of them is the oracle):
* hand-worked runs of Fig. 1 stored under tests/golden/ (with citations);
* closed forms: Manhattan distance on a unit grid, prefix sums on a path
  (numpy cumsum in the weight dtype), star graph, BFS hop counts (scipy);
* scipy.sparse.csgraph.dijkstra (float64, exact for these integer weights);
* a dense numpy min-plus iteration for hop-limited distances;
* brute-force Bellman-Ford and the set/LA forms must all agree bit for bit;
* schedule invariants every correct delta-stepping run satisfies
  (S_i = {v : floor(d(v)/delta) = i}, heavy edges relaxed once each).
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

from paper_1911_06895_amd import graphs as G

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U32_INF = 0xFFFFFFFF


def _load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _graph_from_edges(n, edges, dtype):
    e = np.array(edges, dtype=np.float64).reshape(-1, 3)
    return G.csr_from_edges(n, e[:, 0].astype(np.int64), e[:, 1].astype(np.int64), e[:, 2].astype(dtype),
                            dedup=False, drop_self_loops=False)


def bits(a: np.ndarray) -> np.ndarray:
    """View distances as unsigned integers so equality is bit equality."""
    return a.view({4: np.uint32, 8: np.uint64}[a.dtype.itemsize])


def finite(d: np.ndarray) -> np.ndarray:
    return d != U32_INF if d.dtype == np.uint32 else np.isfinite(d)


def tiny_random_graph(seed: int):
    """Random small graph, sometimes with parallel edges and self-loops."""
    r = G.rng_for(7000 + seed, G.S_STRUCT)
    n = int(r.integers(2, 41))
    m = int(r.integers(0, 4 * n + 1))
    src = r.integers(0, n, size=m)
    dst = r.integers(0, n, size=m)
    kind = ("u32", "f32", "f64")[seed % 3]
    if kind == "u32":
        w = r.integers(1, int(r.choice([3, 20, 1000])) + 1, size=m).astype(np.uint32)
    elif kind == "f32":
        w = np.exp(r.uniform(math.log(1e-2), math.log(1e2), size=m)).astype(np.float32)
    else:
        w = r.uniform(0.01, 10.0, size=m)
    raw = seed % 2 == 0
    g = G.csr_from_edges(n, src, dst, w, dedup=not raw, drop_self_loops=not raw)
    s = int(r.integers(0, n))
    return g, s


def deltas_for(g):
    w = g.w
    if w.size == 0:
        return [1.0]
    out = [float(np.median(w)), float(w.max()), float(w.astype(np.float64).sum()) + 1.0]
    if w.dtype == np.uint32:
        out.append(1.0)
    else:
        out.append(float(w.min()) / 2.0)
        out.append(0.5)  # dyadic
    return out


def pin_golden_worked_example(o) -> list[str]:
    gd = _load_golden("worked_example_u32.json")
    g = _graph_from_edges(gd["n"], gd["edges"], np.uint32)
    want = np.array([U32_INF if x is None else x for x in gd["dist"]], dtype=np.uint32)
    fails = []
    d1, rc1 = o.dijkstra(g, gd["source"])
    if rc1 or not np.array_equal(d1, want):
        fails.append(f"golden dijkstra {d1} != {want}")
    for name, fn in (("la", o.delta_stepping_la), ("sets", o.delta_stepping_sets)):
        d, rc, tr = fn(g, gd["delta"], gd["source"])
        if rc or not np.array_equal(d, want):
            fails.append(f"golden {name} dist {d} != {want}")
        if list(tr["buckets"]) != gd["buckets"] or list(tr["inner"]) != gd["inner_iterations"]:
            fails.append(f"golden {name} buckets/inner {tr['buckets']} {tr['inner']}")
        if [int(x) for x in tr["s_size"]] != [len(s) for s in gd["s_sets"]]:
            fails.append(f"golden {name} |S_i| {tr['s_size']}")
        for i, sset in zip(gd["buckets"], gd["s_sets"]):
            got = sorted(np.nonzero(tr["s_bucket"] == i)[0].tolist())
            if got != sorted(sset):
                fails.append(f"golden {name} S_{i} = {got} != {sset}")
        if tr["light_relax"] != gd["light_relaxations"] or tr["heavy_relax"] != gd["heavy_relaxations"]:
            fails.append(f"golden {name} relaxations {tr['light_relax']} {tr['heavy_relax']}")
        if tr["outer_iters"] != gd["outer_iterations"]:
            fails.append(f"golden {name} outer {tr['outer_iters']}")
    return fails


def pin_golden_fp32(o) -> list[str]:
    gd = _load_golden("fp32_absorption.json")
    g = _graph_from_edges(gd["n"], gd["edges"], np.float32)
    want = np.array(gd["dist"], dtype=np.float32)
    fails = []
    for name, d in (("dijkstra", o.dijkstra(g, 0)[0]), ("bf", o.bellman_ford(g, 0)[0]),
                    ("la", o.delta_stepping_la(g, 4.0, 0)[0]), ("sets", o.delta_stepping_sets(g, 4.0, 0)[0])):
        if not np.array_equal(bits(d), bits(want)):
            fails.append(f"fp32 golden {name}: {d} != {want}")
    if o.certify(g, 0, want) != 0:
        fails.append("fp32 golden: certificate rejects the fp32 answer")
    exact = np.array(gd["dist_exact_real"], dtype=np.float64)
    if o.certify(g, 0, exact.astype(np.float32)) == 0 and not np.array_equal(exact.astype(np.float32), want):
        fails.append("fp32 golden: certificate accepts exact-real distances")
    return fails


def pin_tiny_random_agree(o, count: int = 300) -> list[str]:
    """Dijkstra, LA delta-stepping, set delta-stepping and Bellman-Ford agree bit for bit."""
    fails = []
    for seed in range(count):
        g, s = tiny_random_graph(seed)
        ref, rc0 = o.bellman_ford(g, s)
        d, rc = o.dijkstra(g, s)
        if rc != rc0 or not np.array_equal(bits(d), bits(ref)):
            fails.append(f"seed {seed}: dijkstra != bellman-ford")
        for delta in deltas_for(g):
            for name, fn in (("la", o.delta_stepping_la), ("sets", o.delta_stepping_sets)):
                dd, rcd, tr = fn(g, delta, s)
                if rcd == 4 or tr["late_requests"]:
                    # a heavy request rounding below (i+1)*delta into a closed bucket can
                    # only happen for floating-point weights with a non-dyadic delta
                    continue
                if rcd != rc0 or not np.array_equal(bits(dd), bits(ref)):
                    fails.append(f"seed {seed} delta {delta}: {name} != bellman-ford")
        if len(fails) > 5:
            break
    return fails


def pin_scipy(o) -> list[str]:
    fails = []
    for g, s in ((G.workload("er_n1024_m8192"), 0), (G.rmat_graph(12, 16, cfg=2), 17),
                 (G.grid_graph(32, 32, cfg=3), 0)):
        A = sp.csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
        ref = csg.dijkstra(A, directed=True, indices=s)
        ref = np.where(np.isinf(ref), U32_INF, ref).astype(np.uint32)
        d, rc = o.dijkstra(g, s)
        if rc or not np.array_equal(d, ref):
            fails.append(f"scipy dijkstra mismatch on {g.name}")
        dl, rc, _ = o.delta_stepping_la(g, 32, s)
        if rc or not np.array_equal(dl, ref):
            fails.append(f"scipy vs la mismatch on {g.name}")
    return fails


def pin_closed_forms(o) -> list[str]:
    fails = []
    # unit grid: Manhattan distance from a corner and from an interior vertex
    rows, cols = 17, 23
    g = G.grid_graph(rows, cols, cfg=3, weights="unit_u32")
    for (r0, c0) in ((0, 0), (8, 11)):
        s = r0 * cols + c0
        rr, cc = np.divmod(np.arange(rows * cols), cols)
        want = (np.abs(rr - r0) + np.abs(cc - c0)).astype(np.uint32)
        for name, d in (("dijkstra", o.dijkstra(g, s)[0]), ("la", o.delta_stepping_la(g, 3, s)[0]),
                        ("sets", o.delta_stepping_sets(g, 3, s)[0])):
            if not np.array_equal(d, want):
                fails.append(f"grid manhattan {name} from {(r0, c0)}")
    # path graph: prefix sums in the weight type (numpy cumsum accumulates in order)
    r = G.rng_for(8001, G.S_WEIGHT)
    for dt in (np.uint32, np.float32, np.float64):
        n = 200
        if dt == np.uint32:
            w = r.integers(1, 1000, size=n - 1).astype(np.uint32)
        else:
            w = r.uniform(0.001, 3.0, size=n - 1).astype(dt)
        g = G.path_graph(n, w)
        want = np.concatenate([[0], np.cumsum(w, dtype=dt)]).astype(dt)
        for name, d in (("dijkstra", o.dijkstra(g, 0)[0]), ("la", o.delta_stepping_la(g, 1.0, 0)[0]),
                        ("bf", o.bellman_ford(g, 0)[0])):
            if not np.array_equal(bits(d), bits(want)):
                fails.append(f"path prefix sums {dt.__name__} {name}")
        # from the middle: the first half is unreachable
        d = o.dijkstra(g, n // 2)[0]
        if np.any(finite(d[: n // 2])):
            fails.append(f"path {dt.__name__}: vertices behind the source reached")
    # star: d = w
    w = r.integers(1, 50, size=30).astype(np.uint32)
    g = G.star_graph(31, w)
    d = o.delta_stepping_la(g, 10, 0)[0]
    if not np.array_equal(d, np.concatenate([[0], w]).astype(np.uint32)):
        fails.append("star")
    return fails


def pin_bfs_mode(o) -> list[str]:
    """Unit weights with delta = 1 (the paper's experimental setting): distances are BFS
    hop counts, every edge is light, each bucket is one BFS level settled in one light
    phase (Sec. VI-A setting; Sec. VII remark that delta = 1 behaves like Dijkstra)."""
    fails = []
    base = G.er_graph(400, 900, cfg=11, weights="unit_u32")
    g = G.symmetrize(base)
    A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    s = 3
    hops = csg.shortest_path(A, directed=True, unweighted=True, indices=s)
    want = np.where(np.isinf(hops), U32_INF, hops).astype(np.uint32)
    d, rc, tr = o.delta_stepping_la(g, 1, s)
    if rc or not np.array_equal(d, want):
        fails.append("bfs mode distances")
    reached = want != U32_INF
    levels = int(want[reached].max()) + 1
    if tr["heavy_relax"] != 0 or tr["nbuckets"] != levels or not np.all(tr["inner"] == 1):
        fails.append(f"bfs mode trace: heavy={tr['heavy_relax']} buckets={tr['nbuckets']} inner={tr['inner']}")
    if not np.array_equal(tr["s_bucket"][reached], want[reached].astype(np.int64)):
        fails.append("bfs mode: S_i is not BFS level i")
    if tr["light_relax"] != int(g.outdeg()[reached].sum()):
        fails.append("bfs mode: each reached edge is relaxed once")
    return fails


def _light_heavy_counts(g, d, delta_split):
    src = g.edge_src()
    fin = finite(d)[src]
    wv = g.w.astype(np.float64)
    light = (wv > 0) & (wv <= delta_split)
    return int((fin & light).sum()), int((fin & ~light).sum())


def pin_schedule_invariants(o) -> list[str]:
    """Every correct run: S_i = {v : floor(d/delta) = i}; buckets with a non-empty S are
    exactly the floor(d/delta) values; each reached heavy edge is relaxed exactly once;
    each reached light edge at least once."""
    fails = []
    cases = [(G.er_graph(300, 2400, cfg=12, weights="u32", wlo=1, whi=100), 0, 16),
             (G.er_graph(300, 2400, cfg=13, weights="f32_loguniform", wlo=1e-2, whi=1e2), 5, 0.25),
             (G.grid_graph(12, 12, cfg=14, weights="u32", wlo=1, whi=1000), 0, 100)]
    for g, s, delta in cases:
        dref = o.dijkstra(g, s)[0]
        fin = finite(dref)
        dsplit = float(np.float32(delta)) if g.w.dtype == np.float32 else float(delta)
        want_b = np.array([math.floor(Fraction(float(x)) / Fraction(dsplit)) for x in dref[fin]], dtype=np.int64)
        nl, nh = _light_heavy_counts(g, dref, dsplit)
        for name, fn in (("la", o.delta_stepping_la), ("sets", o.delta_stepping_sets)):
            d, rc, tr = fn(g, delta, s)
            if not np.array_equal(bits(d), bits(dref)):
                fails.append(f"{g.name} {name}: distances")
            if not np.array_equal(tr["s_bucket"][fin], want_b) or np.any(tr["s_bucket"][~fin] != -1):
                fails.append(f"{g.name} {name}: S_i != floor(d/delta)")
            if sorted(tr["buckets"].tolist()) != sorted(set(want_b.tolist())) or tr["s_conflicts"]:
                fails.append(f"{g.name} {name}: non-empty buckets")
            if tr["heavy_relax"] != nh or tr["light_relax"] < nl:
                fails.append(f"{g.name} {name}: relax counts {tr['light_relax']}/{nl} {tr['heavy_relax']}/{nh}")
    return fails


def _hop_limited_depth(g, s):
    """Smallest h such that h-edge-limited distances equal the true distances
    (dense min-plus iteration in numpy, exact for small integer weights)."""
    n = g.n
    W = np.full((n, n), np.inf)
    src = g.edge_src()
    np.minimum.at(W, (src, g.col), g.w.astype(np.float64))
    d = np.full(n, np.inf)
    d[s] = 0.0
    h = 0
    while True:
        nd = np.minimum(d, (d[:, None] + W).min(axis=0))
        if np.array_equal(nd, d):
            return h, d
        d = nd
        h += 1


def pin_special_deltas(o) -> list[str]:
    fails = []
    g = G.er_graph(120, 700, cfg=15, weights="u32", wlo=1, whi=50)
    s = 1
    dref = o.dijkstra(g, s)[0]
    fin = finite(dref)
    # delta >= max w: A_H is empty
    d, _, tr = o.delta_stepping_la(g, 50, s)
    if tr["heavy_relax"] != 0 or not np.array_equal(d, dref):
        fails.append("delta >= max w: heavy phase not empty")
    # delta < min w: A_L is empty, one light phase per bucket
    d, _, tr = o.delta_stepping_la(g, 0.5, s)
    if tr["light_relax"] != 0 or np.any(tr["inner"] != 1) or not np.array_equal(d, dref):
        fails.append("delta < min w: light phase not empty")
    # delta beyond every distance and weight: one bucket = synchronous Bellman-Ford,
    # inner iterations = fewest-hop depth of the shortest-path forest + 1
    h, dd = _hop_limited_depth(g, s)
    if not np.array_equal(np.where(np.isinf(dd), U32_INF, dd).astype(np.uint32), dref):
        fails.append("dense min-plus != dijkstra")
    big = int(dref[fin].max()) + 51
    d, _, tr = o.delta_stepping_la(g, big, s)
    if tr["nbuckets"] != 1 or list(tr["inner"]) != [h + 1] or not np.array_equal(d, dref):
        fails.append(f"single bucket: inner {tr['inner']} != {h + 1}")
    return fails


def pin_certificate(o) -> list[str]:
    """The certificate accepts the exact answer and rejects each kind of wrong answer."""
    fails = []
    for g in (G.er_graph(200, 1200, cfg=16, weights="u32", wlo=1, whi=100),
              G.er_graph(200, 1200, cfg=17, weights="f32_unit")):
        s = int(G.sources_with_outedges(g, 1, cfg=16)[0])
        d = o.dijkstra(g, s)[0]
        if o.certify(g, s, d) != 0:
            fails.append(f"certificate rejects the answer on {g.name}")
        fin = np.nonzero(finite(d))[0]
        fin = fin[fin != s]
        unr = np.nonzero(~finite(d))[0]
        inf = U32_INF if d.dtype == np.uint32 else np.inf
        muts = []
        x = d.copy(); x[fin[0]] = x[fin[0]] + (1 if d.dtype == np.uint32 else np.float32(1e-3)); muts.append(("up", x))
        x = d.copy(); x[fin[1]] = x[fin[1]] - (1 if d.dtype == np.uint32 else np.float32(1e-3)); muts.append(("down", x))
        x = d.copy(); x[fin[2]] = inf; muts.append(("inf", x))
        x = d.copy(); x[s] = 1; muts.append(("source", x))
        if unr.size:
            x = d.copy(); x[unr[0]] = d[fin[3]]; muts.append(("unreachable", x))
        if d.dtype == np.float32:
            x = d.copy(); x[fin[4]] = np.nan; muts.append(("nan", x))
            x = d.copy(); x[s] = -0.0; muts.append(("negzero", x))
        for name, x in muts:
            if o.certify(g, s, x) == 0:
                fails.append(f"certificate accepts mutation {name} on {g.name}")
    return fails


def pin_overflow(o) -> list[str]:
    """u32: 2^32-2 is the largest distance; one more is an overflow. fp32: a sum that
    rounds to +inf is an overflow. All four forms agree."""
    fails = []
    cases = [(np.array([2**31 - 1, 2**31 - 1], dtype=np.uint32), 0),
             (np.array([2**31 - 1, 2**31], dtype=np.uint32), 1),
             (np.array([4_000_000_000, 4_000_000_000], dtype=np.uint32), 1),
             (np.array([3e38, 3e38], dtype=np.float32), 1),
             (np.array([1e38, 1e38], dtype=np.float32), 0)]
    for w, want in cases:
        g = G.path_graph(3, w)
        delta = float(w.max()) / 2  # few buckets: the literal loop steps through every empty one
        rcs = [o.dijkstra(g, 0)[1], o.bellman_ford(g, 0)[1], o.delta_stepping_la(g, delta, 0)[1],
               o.delta_stepping_sets(g, delta, 0)[1]]
        if rcs != [want] * 4:
            fails.append(f"overflow verdicts {rcs} for {w}")
    # an overflowing detour next to a representable path is not an overflow
    g = G.csr_from_edges(3, np.array([0, 0, 1]), np.array([1, 2, 2]),
                         np.array([4_000_000_000, 5, 1_000_000_000], dtype=np.uint32))
    if o.dijkstra(g, 0)[1] != 0 or o.bellman_ford(g, 0)[1] != 0:
        fails.append("overflowing detour flagged")
    return fails


def pin_bucket_of(o) -> list[str]:
    fails = []
    r = G.rng_for(8002, G.S_WEIGHT)
    for _ in range(2000):
        delta = float(np.float32(np.exp(r.uniform(-5, 5))))
        k = int(r.integers(0, 10**6))
        base = float(np.float32(k * delta))
        for t in (base, float(np.nextafter(np.float32(base), np.float32(np.inf))),
                  float(np.nextafter(np.float32(base), np.float32(0)))):
            want = math.floor(Fraction(t) / Fraction(delta))
            if o.bucket_of(t, delta) != want:
                fails.append(f"bucket_of({t}, {delta}) != {want}")
    return fails


ALL_PINS = [pin_golden_worked_example, pin_golden_fp32, pin_tiny_random_agree, pin_scipy, pin_closed_forms,
            pin_bfs_mode, pin_schedule_invariants, pin_special_deltas, pin_certificate, pin_overflow,
            pin_bucket_of]


# ---------------------------------------------------------------- adjoint (dL/dw) pins

def _tree_parents_bruteforce(g, s, d):
    """Parent of every reached v != s (numpy): the smallest-index tight in-edge from a strictly
    closer vertex; vertices tight only through equal-distance in-edges (rounding absorption)
    take, round by round, the smallest-index tight in-edge from a vertex resolved in the
    previous round (round 0: s and every vertex with a strictly-closer parent)."""
    src = g.edge_src()
    fin = finite(d)
    wd = g.w.astype(np.float64)
    dd = d.astype(np.float64)
    if g.w.dtype == np.float32:
        cand = (d[src].astype(np.float32) + g.w).astype(np.float64)
    else:
        cand = dd[src] + wd
    tight = fin[src] & (cand == dd[g.col]) & (g.col != s)
    parent = np.full(g.n, -1, dtype=np.int64)
    strict = tight & (dd[src] < dd[g.col])
    for e in np.nonzero(strict)[0][::-1]:  # descending, so the smallest index is written last
        parent[g.col[e]] = e
    rnd = np.where(fin & ((np.arange(g.n) == s) | (parent >= 0)), 0, -1)
    k = 1
    while True:
        grow = tight & (rnd[src] == k - 1) & (rnd[g.col] < 0)
        if not grow.any():
            break
        for e in np.nonzero(grow)[0][::-1]:
            parent[g.col[e]] = e
        rnd[g.col[grow]] = k
        k += 1
    return parent, src


def pin_gradient_closed_forms(o) -> list[str]:
    fails = []
    r = G.rng_for(8100, G.S_WEIGHT)
    # path 0 -> 1 -> ... -> n-1: d(t) = sum of the first t weights, dL/dw_j = sum_{t > j} c_t
    n = 60
    w = r.uniform(1.0, 2.0, size=n - 1)
    c = r.standard_normal(n)
    g = G.path_graph(n, w)
    d, _ = o.dijkstra(g, 0)
    gw, _ = o.sp_gradient(g, 0, d, c)
    want = np.cumsum(c[::-1])[::-1][1:]
    if not np.allclose(gw, want, rtol=1e-12, atol=1e-12):
        fails.append("adjoint on a path: not the suffix sums of the coefficients")
    # star: dL/dw_(0,t) = c_t
    g = G.star_graph(25, r.uniform(1.0, 2.0, size=24))
    c = r.standard_normal(25)
    d, _ = o.dijkstra(g, 0)
    gw, _ = o.sp_gradient(g, 0, d, c)
    if not np.allclose(gw, c[1:], rtol=0, atol=0):
        fails.append("adjoint on a star")
    # unit coefficients: every tree edge receives the size of the subtree below it (integers),
    # checked by walking each vertex's tree path in Python; non-tree edges receive 0
    for dt in (np.uint32, np.float32, np.float64):
        g = G.er_graph(150, 900, cfg=81, weights="u32", wlo=1, whi=9)
        if dt != np.uint32:
            g = G.Graph(n=g.n, row_ptr=g.row_ptr, col=g.col, w=g.w.astype(dt))
        s = int(G.sources_with_outedges(g, 1, cfg=81)[0])
        d, _ = o.dijkstra(g, s)
        ones = finite(d).astype(np.float64)
        gw, pe = o.sp_gradient(g, s, d, ones)
        parent, src = _tree_parents_bruteforce(g, s, d)
        if not np.array_equal(pe, parent):
            fails.append(f"adjoint parents ({dt.__name__}): not the smallest strictly-closer tight in-edge")
            continue
        want = np.zeros(g.m)
        for t in np.nonzero(finite(d))[0]:
            v = t
            while v != s:
                want[parent[v]] += 1.0
                v = src[parent[v]]
        if not np.array_equal(gw, want):
            fails.append(f"adjoint subtree sizes ({dt.__name__})")
    return fails


def pin_gradient_finite_differences(o) -> list[str]:
    """Central differences (h = 1e-3) of L(w) = sum_s sum_t c_t d_s(t) with float64 weights on
    a 200-vertex instance (continuous weights: shortest paths unique almost surely). Edges whose
    response is not linear over [w - h, w + h] (a path change within h) are skipped."""
    fails = []
    g = G.er_graph(200, 1600, cfg=82, weights="f64", wlo=1.0, whi=2.0)
    srcs = [int(x) for x in G.sources_with_outedges(g, 2, cfg=82)]
    c = G.rng_for(82, G.S_COEF).standard_normal(g.n)

    def loss(wv):
        gg = G.Graph(n=g.n, row_ptr=g.row_ptr, col=g.col, w=wv)
        total = 0.0
        for s in srcs:
            d, _ = o.dijkstra(gg, s)
            fin = np.isfinite(d)
            total += float(np.dot(c[fin], d[fin]))
        return total

    grad = np.zeros(g.m)
    for s in srcs:
        d, _ = o.dijkstra(g, s)
        o.sp_gradient(g, s, d, c, grad)
    h = 1e-3
    l0 = loss(g.w)
    compared = 0
    for e in range(g.m):
        wp = g.w.copy(); wp[e] += h
        wm = g.w.copy(); wm[e] -= h
        lp, lm = loss(wp), loss(wm)
        if abs(lp - 2 * l0 + lm) > 1e-9 * max(1.0, abs(l0)):
            continue
        compared += 1
        fd = (lp - lm) / (2 * h)
        if abs(fd - grad[e]) > 1e-6 * max(1.0, abs(grad[e])):
            fails.append(f"edge {e}: finite difference {fd} vs adjoint {grad[e]}")
            if len(fails) > 5:
                break
    if compared < 0.9 * g.m:
        fails.append(f"only {compared} of {g.m} edges had a linear response")
    return fails


def pin_gradient_ties(o) -> list[str]:
    """Two equal shortest paths to vertex 3: the gradient follows the in-edge of smallest index."""
    g = G.csr_from_edges(4, np.array([0, 0, 1, 2]), np.array([1, 2, 3, 3]),
                         np.array([1.0, 1.0, 1.0, 1.0]), dedup=False)
    d, _ = o.dijkstra(g, 0)
    gw, pe = o.sp_gradient(g, 0, d, np.array([0.0, 0.0, 0.0, 5.0]))
    # edges in CSR order: 0->1 (0), 0->2 (1), 1->3 (2), 2->3 (3); the tie at 3 goes to edge 2
    if pe[3] != 2 or not np.array_equal(gw, [5.0, 0.0, 5.0, 0.0]):
        return [f"tie-break: parent {pe[3]}, grad {gw}"]
    return []


def pin_gradient_absorption(o) -> list[str]:
    """The hand-worked binary32 absorption case (tests/golden/fp32_absorption_adjoint.json): two
    vertices at equal distance whose tight edges form a cycle; the tree goes through the
    strictly closer vertex first."""
    gd = _load_golden("fp32_absorption_adjoint.json")
    g = _graph_from_edges(gd["n"], gd["edges"], np.float32)
    want_d = np.array(gd["dist"], dtype=np.float32)
    fails = []
    d, rc = o.dijkstra(g, gd["source"])
    if rc or not np.array_equal(bits(d), bits(want_d)):
        fails.append(f"absorption golden: distances {d} != {want_d}")
        return fails
    if o.certify(g, gd["source"], want_d) != 0:
        fails.append("absorption golden: certificate rejects the fp32 distances")
    try:
        gw, pe = o.sp_gradient(g, gd["source"], want_d, np.array(gd["grad_dist"], dtype=np.float64))
    except ValueError as e:
        return fails + [f"absorption golden: gradient refused the distances ({e})"]
    if pe.tolist() != gd["parent_edge"] or gw.tolist() != gd["grad_w"]:
        fails.append(f"absorption golden: parents {pe.tolist()} grad {gw.tolist()}")
    parent, _ = _tree_parents_bruteforce(g, gd["source"], want_d)
    if parent.tolist() != gd["parent_edge"]:
        fails.append(f"absorption golden: numpy parents {parent.tolist()}")
    return fails


ALL_PINS += [pin_gradient_closed_forms, pin_gradient_finite_differences, pin_gradient_ties, pin_gradient_absorption]
