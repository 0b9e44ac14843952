"""Seeded synthetic graph generators (inputs only; no shortest-path arithmetic).

Every workload graph is a directed adjacency matrix stored row-wise (CSR): row
``u`` lists the out-edges of vertex ``u``, matching the paper's convention that
the i-th row of A holds the edges leaving v_i (Sec. II, adjacency matrices).
The paper's own inputs (SNAP / GraphChallenge, Sec. VI-A) are not available, so
these seeded families stand in for them:

* ``er``     directed Erdos-Renyi G(n, m): exactly m distinct ordered pairs u != v;
* ``rmat``   recursive R-MAT with quadrant probabilities (a, b, c, d), ids permuted;
* ``grid``   2-D 4-neighbour grid, bidirectional edges (high diameter);
* ``ragged`` many independent ER graphs with log-uniform sizes.

Randomness: numpy ``PCG64(SeedSequence([1911, 6895, cfg, stream]))`` with one
stream per purpose (structure, weights, permutation, sources, targets,
coefficients, sizes), so each quantity is reproducible on its own.

This module is shared by the tests, the benchmark and the oracle checks; it
holds no part of the method itself.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# stream ids of the seed sequence
S_STRUCT, S_WEIGHT, S_PERM, S_SOURCES, S_TARGETS, S_COEF, S_SIZES = range(7)

WEIGHT_U32 = "u32"
WEIGHT_F32 = "f32"
WEIGHT_F64 = "f64"


def rng_for(cfg: int, stream: int) -> np.random.Generator:
    """Seeded generator for (configuration id, purpose stream)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1911, 6895, int(cfg), int(stream)])))


@dataclasses.dataclass
class Graph:
    """CSR of a directed weighted graph. Row u = out-edges of u."""

    n: int
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray  # int32 [m]
    w: np.ndarray  # uint32 | float32 | float64 [m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    @property
    def wtype(self) -> str:
        return {np.dtype(np.uint32): WEIGHT_U32, np.dtype(np.float32): WEIGHT_F32,
                np.dtype(np.float64): WEIGHT_F64}[self.w.dtype]

    def outdeg(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edge_src(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), self.outdeg())

    def check(self) -> None:
        rp = self.row_ptr
        assert rp.dtype == np.int64 and rp.shape == (self.n + 1,)
        assert rp[0] == 0 and rp[-1] == self.m and np.all(np.diff(rp) >= 0)
        assert self.col.dtype == np.int32
        if self.m:
            assert self.col.min() >= 0 and self.col.max() < self.n


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, w: np.ndarray, *, dedup: bool = True,
                   drop_self_loops: bool = True, name: str = "") -> Graph:
    """Build a CSR from an edge list.

    Self-loops are removed and parallel edges collapse to the one of minimum
    weight (a simple graph, as the paper assumes), rows sorted by destination.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if drop_self_loops:
        keep = src != dst
        src, dst, w = src[keep], dst[keep], w[keep]
    key = src * n + dst  # < n^2, row-major order
    if dedup:
        if w.dtype == np.uint32 and n <= (1 << 22) and (w.size == 0 or int(w.max()) < (1 << 20)):
            # pack (key, weight) into one word (key < 2^44): after sorting, the
            # first of each key group carries the minimum weight
            packed = (key.astype(np.uint64) << np.uint64(20)) | w.astype(np.uint64)
            packed.sort()
            k2 = packed >> np.uint64(20)
            first = np.ones(k2.shape, dtype=bool)
            first[1:] = k2[1:] != k2[:-1]
            packed = packed[first]
            key = (packed >> np.uint64(20)).astype(np.int64)
            w = (packed & np.uint64((1 << 20) - 1)).astype(np.uint32)
        else:
            order = np.lexsort((w, key))
            key, w = key[order], w[order]
            first = np.ones(key.shape, dtype=bool)
            first[1:] = key[1:] != key[:-1]
            key, w = key[first], w[first]
    else:
        order = np.argsort(key, kind="stable")
        key, w = key[order], w[order]
    s = (key // n).astype(np.int64) if n else key
    d = (key % n).astype(np.int32) if n else key.astype(np.int32)
    counts = np.bincount(s, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    g = Graph(n=n, row_ptr=row_ptr, col=np.ascontiguousarray(d), w=np.ascontiguousarray(w), name=name)
    return g


# ---------------------------------------------------------------- weights

def weights_uniform_u32(rng: np.random.Generator, size: int, lo: int, hi: int) -> np.ndarray:
    """uint32 weights uniform on the integers [lo, hi]."""
    return rng.integers(lo, hi + 1, size=size, dtype=np.uint32)


def weights_loguniform_f32(rng: np.random.Generator, size: int, lo: float, hi: float) -> np.ndarray:
    """fp32(exp(U[ln lo, ln hi]))."""
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size)).astype(np.float32)


def weights_unit_interval_f32(rng: np.random.Generator, size: int) -> np.ndarray:
    """(k+1)/2^24 with k uniform on {0..2^24-1}: uniform on (0, 1], exact in fp32."""
    k = rng.integers(0, 1 << 24, size=size, dtype=np.int64)
    return ((k + 1).astype(np.float64) / float(1 << 24)).astype(np.float32)


def weights_one_two_f32(rng: np.random.Generator, size: int) -> np.ndarray:
    """1 + k/2^23 with k uniform on {0..2^23-1}: uniform on [1, 2), exact in fp32."""
    k = rng.integers(0, 1 << 23, size=size, dtype=np.int64)
    return (1.0 + k.astype(np.float64) / float(1 << 23)).astype(np.float32)


def weights_uniform_f64(rng: np.random.Generator, size: int, lo: float, hi: float) -> np.ndarray:
    return rng.uniform(lo, hi, size=size)


# ---------------------------------------------------------------- structures

def er_pairs(rng: np.random.Generator, n: int, m: int) -> tuple[np.ndarray, np.ndarray]:
    """Exactly m distinct ordered pairs (u, v), u != v, uniform (rejection sampling)."""
    if m > n * (n - 1):
        raise ValueError("too many edges for a simple directed graph")
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        draw = rng.integers(0, n * n, size=max(16, int(need * 1.2) + 16), dtype=np.int64)
        draw = draw[(draw // n) != (draw % n)]
        # keep first occurrences in draw order, then trim
        allk = np.concatenate([keys, draw])
        _, idx = np.unique(allk, return_index=True)
        idx.sort()
        keys = allk[idx][:m]
    return keys // n, keys % n


def er_pairs_sorted(rng: np.random.Generator, n: int, m: int) -> tuple[np.ndarray, np.ndarray]:
    """Exactly m distinct ordered pairs (u, v), u != v, uniform, in row-major order: the
    distinct values of m draws, topped up by fresh draws until there are m."""
    if m > n * (n - 1):
        raise ValueError("too many edges for a simple directed graph")
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m:
        draw = rng.integers(0, n * n, size=m - keys.size, dtype=np.int64)
        draw = draw[(draw // n) != (draw % n)]
        keys = np.union1d(keys, draw)
    return keys // n, keys % n


def er_graph(n: int, m: int, *, cfg: int, weights: str = "u32", wlo=1, whi=100, name: str = "") -> Graph:
    rs, rw = rng_for(cfg, S_STRUCT), rng_for(cfg, S_WEIGHT)
    src, dst = er_pairs(rs, n, m)
    w = _draw_weights(rw, m, weights, wlo, whi)
    return csr_from_edges(n, src, dst, w, name=name or f"er_n{n}_m{m}")


def _draw_weights(rng, size, kind, lo, hi):
    if kind == "u32":
        return weights_uniform_u32(rng, size, int(lo), int(hi))
    if kind == "f32_loguniform":
        return weights_loguniform_f32(rng, size, lo, hi)
    if kind == "f32_unit":
        return weights_unit_interval_f32(rng, size)
    if kind == "f32_one_two":
        return weights_one_two_f32(rng, size)
    if kind == "f64":
        return weights_uniform_f64(rng, size, lo, hi)
    if kind == "unit_u32":
        return np.ones(size, dtype=np.uint32)
    raise ValueError(kind)


def rmat_pairs(rng: np.random.Generator, scale: int, draws: int, a: float, b: float, c: float,
               chunk: int = 1 << 24) -> tuple[np.ndarray, np.ndarray]:
    """Textbook recursive R-MAT: at each of ``scale`` levels pick quadrant
    (0,0),(0,1),(1,0),(1,1) with probabilities a,b,c,1-a-b-c (no per-level noise)."""
    ta = np.uint32(min(int(a * 2.0**32), 2**32 - 1))
    tab = np.uint32(min(int((a + b) * 2.0**32), 2**32 - 1))
    tabc = np.uint32(min(int((a + b + c) * 2.0**32), 2**32 - 1))
    src = np.zeros(draws, dtype=np.uint32)
    dst = np.zeros(draws, dtype=np.uint32)
    for lo in range(0, draws, chunk):
        hi = min(draws, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.uint32)
        d = np.zeros(hi - lo, dtype=np.uint32)
        for lvl in range(scale):
            r = rng.integers(0, 2**32, size=hi - lo, dtype=np.uint32)
            sbit = r >= tab
            dbit = ((r >= ta) & (r < tab)) | (r >= tabc)
            bit = np.uint32(1 << (scale - 1 - lvl))
            s |= sbit.astype(np.uint32) * bit
            d |= dbit.astype(np.uint32) * bit
        src[lo:hi] = s
        dst[lo:hi] = d
    return src, dst


def rmat_graph(scale: int, edge_factor: int = 16, *, cfg: int, a=0.57, b=0.19, c=0.19,
               weights: str = "u32", wlo=1, whi=255, name: str = "") -> Graph:
    n = 1 << scale
    draws = edge_factor * n
    src, dst = rmat_pairs(rng_for(cfg, S_STRUCT), scale, draws, a, b, c)
    w = _draw_weights(rng_for(cfg, S_WEIGHT), draws, weights, wlo, whi)
    perm = rng_for(cfg, S_PERM).permutation(n).astype(np.uint32)
    src = perm[src]
    dst = perm[dst]
    return csr_from_edges(n, src, dst, w, name=name or f"rmat_s{scale}_ef{edge_factor}")


def grid_graph(rows: int, cols: int, *, cfg: int, weights: str = "u32", wlo=1, whi=1000,
               name: str = "") -> Graph:
    """4-neighbour grid, vertex id r*cols+c, one weight drawn per directed edge."""
    n = rows * cols
    ids = np.arange(n, dtype=np.int64)
    r, c = ids // cols, ids % cols
    cand = []
    for dr, dc in ((-1, 0), (0, -1), (0, 1), (1, 0)):  # sorted by destination id
        ok = (r + dr >= 0) & (r + dr < rows) & (c + dc >= 0) & (c + dc < cols)
        cand.append((ids[ok], ids[ok] + dr * cols + dc))
    src = np.concatenate([s for s, _ in cand])
    dst = np.concatenate([d for _, d in cand])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    w = _draw_weights(rng_for(cfg, S_WEIGHT), src.size, weights, wlo, whi)
    counts = np.bincount(src, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.int32), w=w, name=name or f"grid_{rows}x{cols}")


def ragged_er_batch(count: int, *, cfg: int, nlo=1_000, nhi=100_000, avg_deg=8, weights="f32_unit",
                    wlo=0.0, whi=1.0) -> list[Graph]:
    """Independent directed ER graphs with n_i = round(exp(U[ln nlo, ln nhi])), m_i = avg_deg * n_i."""
    sizes = np.rint(np.exp(rng_for(cfg, S_SIZES).uniform(math.log(nlo), math.log(nhi), size=count))).astype(np.int64)
    rs, rw = rng_for(cfg, S_STRUCT), rng_for(cfg, S_WEIGHT)
    out = []
    for gi, n in enumerate(sizes):
        n = int(n)
        s, d = er_pairs_sorted(rs, n, avg_deg * n)
        w = _draw_weights(rw, s.size, weights, wlo, whi)
        row_ptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(s, minlength=n), out=row_ptr[1:])
        out.append(Graph(n=n, row_ptr=row_ptr, col=d.astype(np.int32), w=w, name=f"ragged{gi}_n{n}"))
    return out


def block_union(graphs: list[Graph], name: str = "") -> tuple[Graph, np.ndarray]:
    """The disjoint union of graphs (block-diagonal adjacency matrix) and the first
    vertex of each block (offsets [len(graphs) + 1])."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum([g.n for g in graphs], out=offs[1:])
    eoffs = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum([g.m for g in graphs], out=eoffs[1:])
    row_ptr = np.concatenate([g.row_ptr[:-1] + eoffs[i] for i, g in enumerate(graphs)] + [eoffs[-1:]])
    col = np.concatenate([g.col.astype(np.int64) + offs[i] for i, g in enumerate(graphs)]).astype(np.int32)
    w = np.concatenate([g.w for g in graphs])
    return Graph(n=int(offs[-1]), row_ptr=row_ptr, col=col, w=w, name=name or f"union{len(graphs)}"), offs


def sources_with_outedges(g: Graph, k: int, *, cfg: int) -> np.ndarray:
    """k distinct sources uniform among vertices with out-degree > 0."""
    cand = np.nonzero(g.outdeg() > 0)[0]
    pick = rng_for(cfg, S_SOURCES).choice(cand.size, size=min(k, cand.size), replace=False)
    return cand[pick].astype(np.int32)


def targets_and_coefs(n: int, k: int, *, cfg: int) -> tuple[np.ndarray, np.ndarray]:
    t = rng_for(cfg, S_TARGETS).choice(n, size=min(k, n), replace=False).astype(np.int32)
    c = rng_for(cfg, S_COEF).standard_normal(t.size).astype(np.float32)
    return t, c


# ---------------------------------------------------------------- small structured graphs for pins

def path_graph(n: int, w: np.ndarray) -> Graph:
    src = np.arange(n - 1)
    return csr_from_edges(n, src, src + 1, np.asarray(w), name=f"path{n}")


def star_graph(n: int, w: np.ndarray) -> Graph:
    src = np.zeros(n - 1, dtype=np.int64)
    return csr_from_edges(n, src, np.arange(1, n), np.asarray(w), name=f"star{n}")


def symmetrize(g: Graph) -> Graph:
    """Undirected version of g (edge in both directions, min weight)."""
    s = g.edge_src().astype(np.int64)
    d = g.col.astype(np.int64)
    return csr_from_edges(g.n, np.concatenate([s, d]), np.concatenate([d, s]), np.concatenate([g.w, g.w]),
                          name=g.name + "_sym")


# ---------------------------------------------------------------- named workloads

def workload(name: str) -> Graph:
    """The named benchmark and test workloads (sizes stated in the names)."""
    if name == "er_n1024_m8192":
        return er_graph(1024, 8192, cfg=1, weights="u32", wlo=1, whi=100)
    if name.startswith("rmat_s") and name.endswith("_u32"):  # rmat_s22_u32
        scale = int(name[len("rmat_s"):].split("_")[0])
        return rmat_graph(scale, 16, cfg=2, weights="u32", wlo=1, whi=255)
    if name.startswith("grid") and name.endswith("_u32"):  # grid4096_u32
        side = int(name[len("grid"):].split("_")[0])
        return grid_graph(side, side, cfg=3, weights="u32", wlo=1, whi=1000)
    if name.startswith("rmat_s") and name.endswith("_f32log"):
        scale = int(name[len("rmat_s"):].split("_")[0])
        return rmat_graph(scale, 16, cfg=41, weights="f32_loguniform", wlo=1e-2, whi=1e2)
    if name.startswith("rmat_s") and name.endswith("_f32onetwo"):
        scale = int(name[len("rmat_s"):].split("_")[0])
        return rmat_graph(scale, 16, cfg=5, weights="f32_one_two")
    raise KeyError(name)
