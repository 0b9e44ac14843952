"""Python binding of the C ABI in include/sssp.h (argument marshalling only).

Every computation runs in libsssp.so (HIP kernels for gfx950); torch supplies
device memory and the current HIP stream. There is no CPU fallback: if the
library is missing, the first call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(_PKG, "libsssp.so")

SSSP_OK = 0
SSSP_ERR_INVALID_ARGUMENT = 1
SSSP_ERR_INVALID_WEIGHT = 2
SSSP_ERR_OUT_OF_MEMORY = 3
SSSP_ERR_DEVICE = 4
SSSP_ERR_OVERFLOW = 5
SSSP_ERR_NO_FORWARD = 6
SSSP_ERR_UNSUPPORTED = 7

SSSP_WEIGHT_U32 = 0
SSSP_WEIGHT_F32 = 1
SSSP_WEIGHT_F64 = 2

EXPORTS = ("sssp_create", "sssp_solve", "sssp_solve_async", "sssp_solve_multi", "sssp_solve_multi_async",
           "sssp_solve_status", "sssp_backward", "sssp_set_weights", "sssp_last_stats", "sssp_set_tuning",
           "sssp_set_trace", "sssp_graph_info", "sssp_destroy", "sssp_status_string", "sssp_autotune",
           "sssp_get_tuning", "sssp_backward_noalloc")


class SsspGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("weights", ctypes.c_void_p), ("wtype", ctypes.c_int32)]


class SsspStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in
                ("sources", "buckets", "light_phases", "heavy_phases", "far_phases", "light_edges", "heavy_edges",
                 "improvements", "attempts", "barriers", "trace_records")]


TUNING_FIELDS = ("workgroups_per_cu", "ring_buckets", "inline_edges", "concurrent_sources", "wait_limit_ms",
                 "hub_edges", "chunk_entries", "inline_entries", "leader_chain")


class SsspTuning(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in TUNING_FIELDS]


class SsspAutotuneResult(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("concurrent_sources", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("ms", ctypes.c_float), ("tuning", SsspTuning)]


class SsspError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {sssp_status_string(status)} ({status})")
        self.status = status


_lib = None


def load_library(path: str = LIBRARY) -> ctypes.CDLL:
    """Load libsssp.so (built by paper_1911_06895_amd.build). Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.sssp_create.argtypes = [ctypes.POINTER(SsspGraph), ctypes.c_double, P, ctypes.POINTER(P)]
    lib.sssp_create.restype = ctypes.c_int
    lib.sssp_solve.argtypes = [P, P, ctypes.c_int32, P, P]
    lib.sssp_solve.restype = ctypes.c_int
    lib.sssp_solve_async.argtypes = [P, P, ctypes.c_int32, P, P]
    lib.sssp_solve_async.restype = ctypes.c_int
    lib.sssp_solve_multi.argtypes = [P, P, ctypes.c_int32, P, P]
    lib.sssp_solve_multi.restype = ctypes.c_int
    lib.sssp_solve_multi_async.argtypes = [P, P, ctypes.c_int32, P, P]
    lib.sssp_solve_multi_async.restype = ctypes.c_int
    lib.sssp_solve_status.argtypes = [P, P]
    lib.sssp_solve_status.restype = ctypes.c_int
    lib.sssp_backward.argtypes = [P, P, ctypes.c_int32, P, P, P, P]
    lib.sssp_backward.restype = ctypes.c_int
    lib.sssp_backward_noalloc.argtypes = [P, P, ctypes.c_int32, P, P, P, P]
    lib.sssp_backward_noalloc.restype = ctypes.c_int
    lib.sssp_set_weights.argtypes = [P, P, P]
    lib.sssp_set_weights.restype = ctypes.c_int
    lib.sssp_last_stats.argtypes = [P, ctypes.POINTER(SsspStats)]
    lib.sssp_last_stats.restype = ctypes.c_int
    lib.sssp_set_tuning.argtypes = [P, ctypes.POINTER(SsspTuning)]
    lib.sssp_set_tuning.restype = ctypes.c_int
    lib.sssp_get_tuning.argtypes = [P, ctypes.POINTER(SsspTuning)]
    lib.sssp_get_tuning.restype = ctypes.c_int
    lib.sssp_set_trace.argtypes = [P, P, ctypes.c_int64]
    lib.sssp_set_trace.restype = ctypes.c_int
    lib.sssp_graph_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.sssp_graph_info.restype = ctypes.c_int
    lib.sssp_destroy.argtypes = [P]
    lib.sssp_destroy.restype = None
    lib.sssp_autotune.argtypes = [ctypes.POINTER(SsspGraph), P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P,
                                  P, ctypes.POINTER(P), ctypes.POINTER(SsspAutotuneResult)]
    lib.sssp_autotune.restype = ctypes.c_int
    lib.sssp_status_string.argtypes = [ctypes.c_int]
    lib.sssp_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _stream(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _check(status: int, what: str):
    if status != SSSP_OK:
        raise SsspError(status, what)


def sssp_status_string(status: int) -> str:
    return load_library().sssp_status_string(int(status)).decode()


def _graph(row_ptr, col_idx, weights) -> SsspGraph:
    import torch

    if weights.dtype == torch.int32 or weights.dtype == torch.uint32:
        wtype = SSSP_WEIGHT_U32
    elif weights.dtype == torch.float32:
        wtype = SSSP_WEIGHT_F32
    elif weights.dtype == torch.float64:
        wtype = SSSP_WEIGHT_F64
    else:
        raise TypeError(f"weights must be uint32 (or int32 bit patterns), float32 or float64, got {weights.dtype}")
    if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32:
        raise TypeError("row_ptr must be int64 and col_idx int32")
    for t in (row_ptr, col_idx, weights):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("graph arrays must be contiguous GPU tensors")
    n = row_ptr.numel() - 1
    m = col_idx.numel()
    if weights.numel() != m:
        raise ValueError("weights and col_idx differ in length")
    return SsspGraph(n=n, m=m, row_ptr=row_ptr.data_ptr(), col_idx=col_idx.data_ptr() if m else None,
                     weights=weights.data_ptr() if m else None, wtype=wtype)


def sssp_create(row_ptr, col_idx, weights, delta: float, stream=None) -> ctypes.c_void_p:
    """row_ptr int64 [n+1], col_idx int32 [m], weights uint32|float32 [m]: torch tensors on the GPU."""
    g = _graph(row_ptr, col_idx, weights)
    h = ctypes.c_void_p()
    _check(load_library().sssp_create(ctypes.byref(g), float(delta), _stream(stream), ctypes.byref(h)),
           "sssp_create")
    return h


def sssp_autotune(row_ptr, col_idx, weights, sources, dist, multi: bool = False, deltas=None, stream=None):
    """Handle with the fastest (delta, concurrent sources, tile schedule) for a sample of host
    sources; dist is GPU scratch ([k, n], or [n] when multi). Returns (handle, result dict; its
    "tuning" entry is the chosen schedule as a dict)."""
    g = _graph(row_ptr, col_idx, weights)
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1))
    if not dist.is_cuda or not dist.is_contiguous() or dist.element_size() != (8 if g.wtype == SSSP_WEIGHT_F64 else 4):
        raise ValueError("dist must be a contiguous GPU tensor of the weights' element size")
    if dist.numel() < (1 if multi else src.size) * g.n:
        raise ValueError("dist is too small")
    d = None if deltas is None else np.ascontiguousarray(np.asarray(deltas, dtype=np.float64))
    h = ctypes.c_void_p()
    res = SsspAutotuneResult()
    _check(load_library().sssp_autotune(ctypes.byref(g), src.ctypes.data_as(ctypes.c_void_p), int(src.size),
                                        1 if multi else 0,
                                        d.ctypes.data_as(ctypes.c_void_p) if d is not None else None,
                                        0 if d is None else int(d.size), ctypes.c_void_p(dist.data_ptr()),
                                        _stream(stream), ctypes.byref(h), ctypes.byref(res)), "sssp_autotune")
    out = {name: getattr(res, name) for name, _ in SsspAutotuneResult._fields_ if name != "tuning"}
    out["tuning"] = {name: int(getattr(res.tuning, name)) for name in TUNING_FIELDS}
    return h, out


def _check_rows(handle, dist, k: int) -> None:
    """The library writes k rows of n distances (4 bytes, 8 for float64 graphs) into dist."""
    n, _, wtype = sssp_graph_info(handle)
    size = 8 if wtype == SSSP_WEIGHT_F64 else 4
    if dist.element_size() != size or dist.numel() < k * n:
        raise ValueError(f"dist must hold [k={k}, n={n}] {size}-byte elements")


def sssp_solve(handle, sources, dist, stream=None) -> None:
    """sources: host ints [k]; dist: GPU tensor [k, n] (uint32/int32 or float32), overwritten."""
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1))
    if not dist.is_cuda or not dist.is_contiguous():
        raise ValueError("dist must be a contiguous GPU tensor")
    _check_rows(handle, dist, src.size)
    _check(load_library().sssp_solve(handle, src.ctypes.data_as(ctypes.c_void_p), int(src.size),
                                     ctypes.c_void_p(dist.data_ptr()), _stream(stream)), "sssp_solve")


def sssp_solve_async(handle, sources, dist, stream=None) -> None:
    """Enqueue only (capturable): sources is a GPU int32 tensor [k], dist a GPU tensor [k, n]."""
    import torch

    if not sources.is_cuda or sources.dtype != torch.int32 or not sources.is_contiguous():
        raise ValueError("sources must be a contiguous int32 GPU tensor")
    if not dist.is_cuda or not dist.is_contiguous():
        raise ValueError("dist must be a contiguous GPU tensor")
    k = int(sources.numel())
    _check_rows(handle, dist, k)
    _check(load_library().sssp_solve_async(handle, ctypes.c_void_p(sources.data_ptr()), k,
                                           ctypes.c_void_p(dist.data_ptr()), _stream(stream)), "sssp_solve_async")


def sssp_solve_multi(handle, sources, dist, stream=None) -> None:
    """Distances from the nearest of the host sources into dist (GPU [n] of the weight type)."""
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1))
    if not dist.is_cuda or not dist.is_contiguous():
        raise ValueError("dist must be a contiguous GPU tensor")
    _check_rows(handle, dist, 1)
    _check(load_library().sssp_solve_multi(handle, src.ctypes.data_as(ctypes.c_void_p), int(src.size),
                                           ctypes.c_void_p(dist.data_ptr()), _stream(stream)), "sssp_solve_multi")


def sssp_solve_multi_async(handle, sources, dist, stream=None) -> None:
    """Enqueue only: sources a GPU int32 tensor [k], dist a GPU tensor [n]."""
    import torch

    if not sources.is_cuda or sources.dtype != torch.int32 or not sources.is_contiguous():
        raise ValueError("sources must be a contiguous int32 GPU tensor")
    if not dist.is_cuda or not dist.is_contiguous():
        raise ValueError("dist must be a contiguous GPU tensor")
    _check_rows(handle, dist, 1)
    _check(load_library().sssp_solve_multi_async(handle, ctypes.c_void_p(sources.data_ptr()), int(sources.numel()),
                                                 ctypes.c_void_p(dist.data_ptr()), _stream(stream)),
           "sssp_solve_multi_async")


def sssp_solve_status(handle, stream=None) -> None:
    """Wait for the last enqueued solve and raise SsspError if it failed."""
    _check(load_library().sssp_solve_status(handle, _stream(stream)), "sssp_solve_status")


def _check_adjoint_args(handle, k, dist, grad_dist, grad_w) -> None:
    import torch

    for t in (dist, grad_dist, grad_w):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("dist, grad_dist and grad_w must be contiguous GPU tensors")
    n, m, _ = sssp_graph_info(handle)
    _check_rows(handle, dist, k)
    if grad_dist.dtype != torch.float32 or grad_dist.numel() < k * n:
        raise ValueError(f"grad_dist must hold [k={k}, n={n}] float32 elements")
    if grad_w.dtype != torch.float32 or grad_w.numel() < m:
        raise ValueError(f"grad_w must hold m={m} float32 elements")


def sssp_backward(handle, sources, dist, grad_dist, grad_w, stream=None) -> None:
    """dL/dw into grad_w (GPU float32 [m], caller edge order) for dL/ddist = grad_dist ([k, n])."""
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1))
    _check_adjoint_args(handle, int(src.size), dist, grad_dist, grad_w)
    _check(load_library().sssp_backward(handle, src.ctypes.data_as(ctypes.c_void_p), int(src.size),
                                        ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(grad_dist.data_ptr()),
                                        ctypes.c_void_p(grad_w.data_ptr()), _stream(stream)), "sssp_backward")


def sssp_backward_noalloc(handle, sources, dist, grad_dist, grad_w, stream=None) -> None:
    """sssp_backward with the working set in the library's static device array; ``sources`` is a
    GPU int32 tensor [k] (nothing is allocated or staged by the call)."""
    import torch

    if not sources.is_cuda or sources.dtype != torch.int32 or not sources.is_contiguous():
        raise ValueError("sources must be a contiguous GPU int32 tensor")
    k = int(sources.numel())
    _check_adjoint_args(handle, k, dist, grad_dist, grad_w)
    _check(load_library().sssp_backward_noalloc(handle, ctypes.c_void_p(sources.data_ptr()), k,
                                                ctypes.c_void_p(dist.data_ptr()),
                                                ctypes.c_void_p(grad_dist.data_ptr()),
                                                ctypes.c_void_p(grad_w.data_ptr()), _stream(stream)),
           "sssp_backward_noalloc")


def sssp_set_weights(handle, weights, stream=None) -> None:
    """weights: contiguous GPU tensor [m] of the handle's weight type (uint32 as int32 bits, or float32)."""
    if not weights.is_cuda or not weights.is_contiguous():
        raise ValueError("weights must be a contiguous GPU tensor")
    _check(load_library().sssp_set_weights(handle, ctypes.c_void_p(weights.data_ptr() if weights.numel() else 0),
                                           _stream(stream)), "sssp_set_weights")


def sssp_last_stats(handle) -> dict:
    st = SsspStats()
    _check(load_library().sssp_last_stats(handle, ctypes.byref(st)), "sssp_last_stats")
    return {name: int(getattr(st, name)) for name, _ in SsspStats._fields_}


def sssp_set_tuning(handle, **fields) -> None:
    """Schedule parameters (sssp_tuning); omitted fields are 0 (the library default)."""
    unknown = set(fields) - set(TUNING_FIELDS)
    if unknown:
        raise TypeError(f"unknown tuning fields {sorted(unknown)}")
    t = SsspTuning(**{k: int(v) for k, v in fields.items()})
    _check(load_library().sssp_set_tuning(handle, ctypes.byref(t)), "sssp_set_tuning")


def sssp_get_tuning(handle) -> dict:
    """The handle's schedule parameters with every default resolved (sssp_get_tuning)."""
    t = SsspTuning()
    _check(load_library().sssp_get_tuning(handle, ctypes.byref(t)), "sssp_get_tuning")
    return {name: int(getattr(t, name)) for name in TUNING_FIELDS}


def sssp_set_trace(handle, buffer, capacity: int) -> None:
    """buffer: GPU int64/uint64 tensor with at least 4 * capacity elements (or None)."""
    ptr = ctypes.c_void_p(buffer.data_ptr()) if buffer is not None and capacity > 0 else None
    _check(load_library().sssp_set_trace(handle, ptr, int(capacity) if ptr is not None else 0), "sssp_set_trace")


ACTIONS = {1: "light", 2: "heavy", 3: "far", 4: "done", 5: "overflow-check", 6: "hub"}


def decode_trace(words, records: int, clock_khz: float) -> list[dict]:
    """Step records as dicts: duration in microseconds, entries, edges scanned, distances lowered."""
    w = np.asarray(words, dtype=np.uint64).reshape(-1, 4)[:records]
    out = []
    for k in range(len(w) - 1):
        what = int(w[k, 1])
        out.append({"action": ACTIONS.get(what & 0x7F, str(what & 0x7F)), "inline": bool(what & 0x80),
                    "bucket": (what >> 8) & 0xFFFFFF, "entries": what >> 32,
                    "edges": int(w[k + 1, 2]), "improved": int(w[k + 1, 3]),
                    "us": float(int(w[k + 1, 0]) - int(w[k, 0])) * 1e3 / clock_khz})
    return out


def sssp_graph_info(handle) -> tuple[int, int, int]:
    n, m, w = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check(load_library().sssp_graph_info(handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(w)),
           "sssp_graph_info")
    return n.value, m.value, w.value


def sssp_destroy(handle) -> None:
    if handle:
        load_library().sssp_destroy(handle)


class DeltaStepping:
    """Owns a handle for one graph and delta; graph given as numpy CSR arrays."""

    def __init__(self, row_ptr: np.ndarray, col: np.ndarray, w: np.ndarray, delta: float, device="cuda"):
        import torch

        self.torch = torch
        if w.dtype == np.uint32:
            wt = torch.from_numpy(w.view(np.int32)).to(device)
            self.out_dtype = torch.int32  # uint32 bit patterns
        elif w.dtype in (np.float32, np.float64):
            wt = torch.from_numpy(w).to(device)
            self.out_dtype = wt.dtype
        else:
            raise TypeError(f"unsupported weight dtype {w.dtype}")
        rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.int64)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).to(device)
        self.n = int(row_ptr.shape[0] - 1)
        self.m = int(col.shape[0])
        self.device = device
        self.handle = sssp_create(rp, ci, wt, delta)
        self.weights_version = 0  # bumped by every set_weights (the autograd wrapper checks it)
        torch.cuda.synchronize()

    def solve(self, sources, out=None):
        src = np.asarray(sources, dtype=np.int32).reshape(-1)
        if out is None:
            out = self.torch.empty((src.size, self.n), dtype=self.out_dtype, device=self.device)
        sssp_solve(self.handle, src, out)
        return out

    def solve_multi(self, sources, out=None):
        """Distances from the nearest source (GPU tensor [n])."""
        if out is None:
            out = self.torch.empty(self.n, dtype=self.out_dtype, device=self.device)
        sssp_solve_multi(self.handle, sources, out)
        return out

    def solve_numpy(self, sources) -> np.ndarray:
        d = self.solve(sources).cpu().numpy()
        return d.view(np.uint32) if self.out_dtype == self.torch.int32 else d

    def stats(self) -> dict:
        return sssp_last_stats(self.handle)

    def set_weights(self, w) -> None:
        """New weights for the same structure (numpy or GPU tensor, caller edge order)."""
        if isinstance(w, np.ndarray):
            w = self.torch.from_numpy(w.view(np.int32) if w.dtype == np.uint32 else w).to(self.device)
        sssp_set_weights(self.handle, w.contiguous())
        self.weights_version += 1

    def backward(self, sources, dist, grad_dist):
        """dL/dw (float32 [m]) for dL/ddist = grad_dist, dist from solve(sources)."""
        grad_w = self.torch.empty(self.m, dtype=self.torch.float32, device=self.device)
        sssp_backward(self.handle, sources, dist.contiguous(), grad_dist.contiguous().float(), grad_w)
        return grad_w

    def set_tuning(self, **kw):
        sssp_set_tuning(self.handle, **kw)

    def close(self):
        if self.handle:
            sssp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shortest_paths(w, solver: DeltaStepping, sources):
    """Differentiable distances: dist = SSSP(w) from ``sources`` ([k, n], float32), with
    dL/dw computed by the shortest-path-tree adjoint (sssp_backward) in the backward pass.
    ``w`` is a float32 GPU tensor [m] in the caller's edge order; the solver's weights are
    replaced by it (sssp_set_weights) before the solve. The weights are saved for the
    backward pass (torch rejects a backward after an in-place change of ``w``); when the
    solver has been given other weights since this forward pass (another forward on the
    same solver), the backward pass puts these weights back and solves again before the
    adjoint, so every node differentiates its own forward."""
    import torch

    src = [int(x) for x in np.asarray(sources, dtype=np.int64).reshape(-1)]

    class _Sssp(torch.autograd.Function):
        @staticmethod
        def forward(ctx, weights):
            solver.set_weights(weights.detach())
            dist = solver.solve(src)
            ctx.version = solver.weights_version
            ctx.save_for_backward(weights, dist)
            return dist

        @staticmethod
        def backward(ctx, grad_dist):
            weights, dist = ctx.saved_tensors
            if solver.weights_version != ctx.version:
                solver.set_weights(weights.detach())
                again = solver.solve(src)
                if not torch.equal(again.view(torch.int32), dist.view(torch.int32)):
                    raise RuntimeError("shortest_paths: the forward distances cannot be reproduced")
            return solver.backward(src, dist, grad_dist)

    return _Sssp.apply(w)
