"""CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It wraps ``oracle.c`` (plain C, built with gcc) through
ctypes and shares no code with the GPU library.

Functions (each a plain, slow, obviously correct reading of the paper):
  dijkstra(g, s)               textbook binary-heap Dijkstra: the definition of the result
  dijkstra_many(g, ss, t)      dijkstra from many sources on t host threads (CPU-baseline timing)
  delta_stepping_la(g, d, s)   linear-algebra delta-stepping of Fig. 1 (left), with a trace
  delta_stepping_sets(g, d, s) Meyer-Sanders bucket form of Fig. 1 (right), with a trace
  bellman_ford(g, s)           brute force, exact integer sums
  certify(g, s, dist)          O(m) optimality certificate (feasibility + tight-edge reachability)
  sp_gradient(g, s, dist, gd)  dL/dw by reverse accumulation over the shortest-path tree
  bucket_of(t, delta)          exact floor(t / delta)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-pthread", "-Wall", "-Wno-maybe-uninitialized"]

KIND = {np.dtype(np.uint32): 0, np.dtype(np.float32): 1, np.dtype(np.float64): 2}
OK, OVERFLOW, BADARG, NOMEM, CLOSED_BUCKET = 0, 1, 2, 3, 4
CERT_OK, CERT_SOURCE, CERT_VALUE, CERT_FEASIBLE, CERT_OVERFLOW, CERT_TIGHT = range(6)

U32_INF = np.uint32(0xFFFFFFFF)


def compile_source(src_path: str, out_path: str) -> str:
    tmp = out_path + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src_path, "-lm"])
    os.replace(tmp, out_path)
    return out_path


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, no fast-math, no contraction)."""
    if force or not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
        compile_source(SOURCE, LIBRARY)
    return LIBRARY


class Trace(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("nbuckets", ctypes.c_int64), ("bucket", ctypes.c_void_p),
                ("s_size", ctypes.c_void_p), ("inner", ctypes.c_void_p), ("outer_iters", ctypes.c_int64),
                ("light_relax", ctypes.c_int64), ("heavy_relax", ctypes.c_int64),
                ("late_requests", ctypes.c_int64), ("s_bucket", ctypes.c_void_p),
                ("s_conflicts", ctypes.c_int64)]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w)
    if w.dtype not in KIND:
        raise TypeError(f"unsupported weight dtype {w.dtype}")
    return rp, col, w, KIND[w.dtype]


class Oracle:
    """One loaded build of oracle.c (the default one, or a test-built variant)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        for fn in ("orc_dijkstra", "orc_bellman_ford"):
            getattr(lib, fn).argtypes = [I64, P, P, P, ctypes.c_int, ctypes.c_int32, P]
            getattr(lib, fn).restype = ctypes.c_int
        for fn in ("orc_delta_la", "orc_delta_sets"):
            getattr(lib, fn).argtypes = [I64, P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int32, P,
                                         ctypes.POINTER(Trace)]
            getattr(lib, fn).restype = ctypes.c_int
        lib.orc_certify.argtypes = [I64, P, P, P, ctypes.c_int, ctypes.c_int32, P]
        lib.orc_certify.restype = ctypes.c_int
        lib.orc_bucket_of.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_bucket_of.restype = ctypes.c_int64
        lib.orc_sp_gradient.argtypes = [I64, P, P, P, ctypes.c_int, ctypes.c_int32, P, P, P, P]
        lib.orc_sp_gradient.restype = ctypes.c_int
        lib.orc_dijkstra_many.argtypes = [I64, P, P, P, ctypes.c_int, P, ctypes.c_int32, P, ctypes.c_int32]
        lib.orc_dijkstra_many.restype = ctypes.c_int
        self.lib = lib

    def dijkstra(self, g, src: int) -> tuple[np.ndarray, int]:
        """Distances from ``src`` in the weights' dtype (unreachable = 2^32-1 / +inf) and a status."""
        rp, col, w, kind = _csr(g)
        out = np.empty(g.n, dtype=w.dtype)
        rc = self.lib.orc_dijkstra(g.n, _ptr(rp), _ptr(col), _ptr(w), kind, int(src), _ptr(out))
        if rc == BADARG:
            raise ValueError("bad graph or source")
        return out, rc

    def dijkstra_many(self, g, sources, threads: int) -> tuple[np.ndarray, int]:
        """dijkstra for every source (rows of the result), run on ``threads`` host threads."""
        rp, col, w, kind = _csr(g)
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1))
        if src.size and (src.min() < 0 or src.max() >= g.n):
            raise ValueError("bad source")
        out = np.empty((src.size, g.n), dtype=w.dtype)
        rc = self.lib.orc_dijkstra_many(g.n, _ptr(rp), _ptr(col), _ptr(w), kind, _ptr(src), int(src.size),
                                        _ptr(out), int(threads))
        if rc == BADARG:
            raise ValueError("bad graph or source")
        return out, rc

    def bellman_ford(self, g, src: int) -> tuple[np.ndarray, int]:
        rp, col, w, kind = _csr(g)
        out = np.empty(g.n, dtype=w.dtype)
        rc = self.lib.orc_bellman_ford(g.n, _ptr(rp), _ptr(col), _ptr(w), kind, int(src), _ptr(out))
        if rc == BADARG:
            raise ValueError("bad graph or source")
        return out, rc

    def _delta(self, fn_name, g, delta, src):
        rp, col, w, kind = _csr(g)
        out = np.empty(g.n, dtype=w.dtype)
        cap = 1 << 16
        bucket = np.zeros(cap, dtype=np.int64)
        s_size = np.zeros(cap, dtype=np.int64)
        inner = np.zeros(cap, dtype=np.int64)
        s_bucket = np.zeros(g.n, dtype=np.int64)
        tr = Trace(cap=cap, bucket=bucket.ctypes.data, s_size=s_size.ctypes.data, inner=inner.ctypes.data,
                   s_bucket=s_bucket.ctypes.data)
        rc = getattr(self.lib, fn_name)(g.n, _ptr(rp), _ptr(col), _ptr(w), kind, float(delta), int(src),
                                        _ptr(out), ctypes.byref(tr))
        if rc == BADARG:
            raise ValueError("bad graph, delta or source")
        nb = min(tr.nbuckets, cap)
        trace = dict(buckets=bucket[:nb].copy(), s_size=s_size[:nb].copy(), inner=inner[:nb].copy(),
                     nbuckets=tr.nbuckets, outer_iters=tr.outer_iters, light_relax=tr.light_relax,
                     heavy_relax=tr.heavy_relax, late_requests=tr.late_requests, s_bucket=s_bucket,
                     s_conflicts=tr.s_conflicts)
        return out, rc, trace

    def delta_stepping_la(self, g, delta: float, src: int):
        """Literal linear-algebra delta-stepping (Fig. 1 left). Returns (dist, status, trace)."""
        return self._delta("orc_delta_la", g, delta, src)

    def delta_stepping_sets(self, g, delta: float, src: int):
        """Meyer-Sanders bucket form (Fig. 1 right). Returns (dist, status, trace)."""
        return self._delta("orc_delta_sets", g, delta, src)

    def certify(self, g, src: int, dist: np.ndarray) -> int:
        """CERT_OK if ``dist`` is the exact shortest-path vector from ``src``, else a CERT_* code."""
        rp, col, w, kind = _csr(g)
        d = np.ascontiguousarray(dist, dtype=w.dtype)
        rc = self.lib.orc_certify(g.n, _ptr(rp), _ptr(col), _ptr(w), kind, int(src), _ptr(d))
        if rc < 0:
            raise ValueError("bad graph or source")
        return rc

    def bucket_of(self, t: float, delta: float) -> int:
        return int(self.lib.orc_bucket_of(float(t), float(delta)))

    def sp_gradient(self, g, src: int, dist: np.ndarray, grad_dist: np.ndarray, grad_w: np.ndarray | None = None):
        """Accumulate dL/dw (float64 [m], caller edge order) for L = sum grad_dist * dist over the
        shortest-path tree from ``src``; returns (grad_w, parent_edge int64 [n])."""
        rp, col, w, kind = _csr(g)
        d = np.ascontiguousarray(dist, dtype=w.dtype)
        gd = np.ascontiguousarray(grad_dist, dtype=np.float64)
        if grad_w is None:
            grad_w = np.zeros(g.m, dtype=np.float64)
        pe = np.empty(g.n, dtype=np.int64)
        rc = self.lib.orc_sp_gradient(g.n, _ptr(rp), _ptr(col), _ptr(w), kind, int(src), _ptr(d), _ptr(gd),
                                      _ptr(grad_w), _ptr(pe))
        if rc != OK:
            raise ValueError(f"sp_gradient: distances are not a shortest-path vector ({rc})")
        return grad_w, pe


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
            build(force=True)
        _default = Oracle(LIBRARY)
    return _default


def dijkstra(g, src):
    return default().dijkstra(g, src)


def dijkstra_many(g, sources, threads):
    return default().dijkstra_many(g, sources, threads)


def bellman_ford(g, src):
    return default().bellman_ford(g, src)


def delta_stepping_la(g, delta, src):
    return default().delta_stepping_la(g, delta, src)


def delta_stepping_sets(g, delta, src):
    return default().delta_stepping_sets(g, delta, src)


def certify(g, src, dist):
    return default().certify(g, src, dist)


def bucket_of(t, delta):
    return default().bucket_of(t, delta)


def sp_gradient(g, src, dist, grad_dist, grad_w=None):
    return default().sp_gradient(g, src, dist, grad_dist, grad_w)


def reached_edges(g, dist: np.ndarray) -> int:
    """Edges out of reached vertices: the edges every correct solve must examine."""
    inf = U32_INF if dist.dtype == np.uint32 else np.inf
    return int(g.outdeg()[dist != inf].sum())
