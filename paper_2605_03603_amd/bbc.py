"""Python binding of libbbc (include/bbc.h): argument marshalling only.

Every count runs in the HIP library; this module converts numpy arrays or
torch tensors to pointers and status codes to exceptions. Torch supplies
device memory and streams (a CUDA/HIP tensor is passed as a device pointer
with BBC_IN_DEVICE_PTRS; a torch stream can be the context's stream).

If libbbc.so is missing the import of this module raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BBC_LIBRARY", os.path.join(_HERE, "libbbc.so"))

BBC_OK = 0
STATUS_NAMES = {0: "BBC_OK", 1: "BBC_E_INVAL", 2: "BBC_E_RANGE", 3: "BBC_E_SIGN",
                4: "BBC_E_DUP_EDGE", 5: "BBC_E_NOMEM", 6: "BBC_E_OVERFLOW",
                7: "BBC_E_UNSUPPORTED", 8: "BBC_E_NOT_READY", 9: "BBC_E_UNKNOWN_TICKET",
                10: "BBC_E_HIP"}
BBC_E_NOT_READY = 8

BBC_IN_DEVICE_PTRS = 1 << 0
BBC_SIGNS_2BIT_PACKED = 1 << 1
BBC_SIGNS_01 = 1 << 2
BBC_ANCHOR_U = 1 << 4
BBC_ANCHOR_V = 1 << 5
BBC_ANCHOR_SMALLER = 1 << 6

EXPORTED = ["bbc_ctx_create", "bbc_ctx_destroy", "bbc_build_csr", "bbc_build_csr_batch",
            "bbc_graph_free", "bbc_get_graph_info", "bbc_count_global", "bbc_count_per_vertex",
            "bbc_count_through_edges", "bbc_top_vertices", "bbc_count_bbwc",
            "bbc_count_batch", "bbc_submit", "bbc_submit_coo", "bbc_poll", "bbc_wait",
            "bbc_count_global_noalloc", "bbc_get_last_stats", "bbc_set_timing",
            "bbc_set_test_hook", "bbc_get_memory_stats",
            "bbc_status_string", "bbc_last_error"]

BBC_HOOK_NO_WINDOW_TIER = 1
BBC_HOOK_PRELOAD_COUNT = 2
BBC_HOOK_LAUNCH_SHAPE = 3


def launch_shape(chunk_base: int, grid_t_per_cu: int, grid_a_per_cu: int = 2) -> int:
    """Value of BBC_HOOK_LAUNCH_SHAPE for a unit column base, triplet and
    tier-A workgroups per compute unit."""
    return chunk_base | (grid_t_per_cu << 32) | (grid_a_per_cu << 40)


class BBCError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.name}: {detail}" if detail else self.name)


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_u", ctypes.c_uint32), ("n_v", ctypes.c_uint32), ("n_edges", ctypes.c_uint64),
                ("anchor_side", ctypes.c_int32), ("device_bytes", ctypes.c_uint64)]


class CountStats(ctypes.Structure):
    _fields_ = [("active_anchors", ctypes.c_uint64), ("virtual_candidates", ctypes.c_uint64),
                ("pair_units", ctypes.c_uint64), ("candidate_pairs", ctypes.c_uint64),
                ("mask_words", ctypes.c_uint64), ("wedges", ctypes.c_uint64),
                ("pair_words", ctypes.c_uint64), ("ms_build", ctypes.c_float),
                ("ms_pair", ctypes.c_float), ("ms_plan", ctypes.c_float),
                ("ms_triplet", ctypes.c_float), ("attempts", ctypes.c_uint32),
                ("deferred_b", ctypes.c_uint32), ("deferred_c", ctypes.c_uint32),
                ("deferred_d", ctypes.c_uint32), ("deferred_a", ctypes.c_uint32),
                ("deferred_r", ctypes.c_uint32)]


class MemoryStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "cap_bytes", "reserved_bytes", "peak_reserved_bytes", "live_bytes", "serve_admitted_bytes",
        "serve_peak_admitted_bytes", "serve_queued", "serve_peak_queued")]


_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int


def _load(path: str = LIB_PATH) -> ctypes.CDLL:
    # torch ships its own HIP runtime under the same soname as the system one
    # libbbc.so links: whichever is loaded first serves the whole process, and
    # torch needs its own, so it is loaded before the library when present
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(f"libbbc.so not found at {path}; build it with "
                          "`python -m paper_2605_03603_amd.build` (there is no CPU fallback)")
    L = ctypes.CDLL(path)
    L.bbc_status_string.restype = ctypes.c_char_p
    L.bbc_status_string.argtypes = [_i32]
    L.bbc_last_error.restype = ctypes.c_char_p
    L.bbc_last_error.argtypes = [_vp]
    L.bbc_ctx_create.argtypes = [_i32, _vp, _u64, ctypes.POINTER(_vp)]
    L.bbc_ctx_destroy.argtypes = [_vp]
    L.bbc_ctx_destroy.restype = None
    L.bbc_build_csr.argtypes = [_vp, _u32, _u32, _u64, _vp, _vp, _vp, _u32, ctypes.POINTER(_vp)]
    L.bbc_build_csr_batch.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _u32, _vp]
    L.bbc_graph_free.argtypes = [_vp, _vp]
    L.bbc_get_graph_info.argtypes = [_vp, _vp, ctypes.POINTER(GraphInfo)]
    L.bbc_count_global.argtypes = [_vp, _vp, _i32, _i32, ctypes.POINTER(ctypes.c_int64)]
    L.bbc_count_global_noalloc.argtypes = [_vp, _vp, _i32, _i32, ctypes.POINTER(ctypes.c_int64)]
    L.bbc_count_per_vertex.argtypes = [_vp, _vp, _i32, _i32, _i32, _vp,
                                       ctypes.POINTER(ctypes.c_int64)]
    L.bbc_count_through_edges.argtypes = [_vp, _vp, _u64, _vp, _vp, _vp, _vp]
    L.bbc_top_vertices.argtypes = [_vp, _vp, _i32, _u32, _vp, _vp, ctypes.POINTER(_u32)]
    L.bbc_count_bbwc.argtypes = [_vp, _vp, _i32, _i32, ctypes.POINTER(ctypes.c_int64)]
    L.bbc_count_batch.argtypes = [_vp, _vp, _u32, _vp]
    L.bbc_submit.argtypes = [_vp, _vp, ctypes.POINTER(_u64)]
    L.bbc_submit_coo.argtypes = [_vp, _u32, _u32, _u64, _vp, _vp, _vp, _u32, ctypes.POINTER(_u64)]
    L.bbc_poll.argtypes = [_vp, _u64, ctypes.POINTER(ctypes.c_int64)]
    L.bbc_wait.argtypes = [_vp, _u64, ctypes.POINTER(ctypes.c_int64)]
    L.bbc_get_last_stats.argtypes = [_vp, ctypes.POINTER(CountStats)]
    L.bbc_set_timing.argtypes = [_vp, _i32]
    L.bbc_set_test_hook.argtypes = [_vp, _i32, ctypes.c_int64]
    L.bbc_get_memory_stats.argtypes = [_vp, ctypes.POINTER(MemoryStats)]
    for name in EXPORTED:
        fn = getattr(L, name)
        if name not in ("bbc_status_string", "bbc_last_error", "bbc_ctx_destroy"):
            fn.restype = _i32
    return L


lib = _load()


def status_string(s: int) -> str:
    return lib.bbc_status_string(s).decode()


def _ptr(a):
    """(pointer, is_device) of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None, False
    if hasattr(a, "data_ptr"):   # torch tensor
        return ctypes.c_void_p(a.data_ptr()), bool(getattr(a, "is_cuda", False))
    a = np.ascontiguousarray(a)
    return a.ctypes.data_as(ctypes.c_void_p), False


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


class Graph:
    def __init__(self, ctx: "Context", handle: int):
        self.ctx = ctx
        self.handle = ctypes.c_void_p(handle)

    def info(self) -> GraphInfo:
        out = GraphInfo()
        self.ctx._check(lib.bbc_get_graph_info(self.ctx.handle, self.handle, ctypes.byref(out)))
        return out

    def free(self):
        if self.handle and self.ctx.handle:
            lib.bbc_graph_free(self.ctx.handle, self.handle)
        self.handle = None


class Context:
    """A libbbc context on one device (bbc_ctx_create)."""

    def __init__(self, device: int = 0, stream=None, mem_cap: int = 0):
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        h = ctypes.c_void_p()
        st = lib.bbc_ctx_create(device, ctypes.c_void_p(stream) if stream else None, mem_cap,
                                ctypes.byref(h))
        if st != BBC_OK:
            raise BBCError(st, "bbc_ctx_create")
        self.handle = h
        self._keep = []

    def _check(self, st: int):
        if st != BBC_OK:
            raise BBCError(st, lib.bbc_last_error(self.handle).decode())

    def close(self):
        if self.handle:
            lib.bbc_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- building
    def build_csr(self, n_u: int, n_v: int, eu, ev, sign, flags: int = 0) -> Graph:
        m = int(eu.shape[0]) if hasattr(eu, "shape") else len(eu)
        if not hasattr(eu, "data_ptr"):
            eu, ev = _host(eu, np.uint32), _host(ev, np.uint32)
            if not (flags & BBC_SIGNS_2BIT_PACKED):
                sign = _host(sign, np.int8)
            else:
                sign = _host(sign, np.uint8)
        pe, dev = _ptr(eu)
        pv, _ = _ptr(ev)
        ps, _ = _ptr(sign)
        if dev:
            flags |= BBC_IN_DEVICE_PTRS
        out = ctypes.c_void_p()
        self._check(lib.bbc_build_csr(self.handle, n_u, n_v, m, pe, pv, ps, flags, ctypes.byref(out)))
        return Graph(self, out.value)

    def build_csr_batch(self, n_u, n_v, edge_offsets, eu, ev, sign, flags: int = 0) -> List[Graph]:
        n_u = _host(n_u, np.uint32)
        n_v = _host(n_v, np.uint32)
        off = _host(edge_offsets, np.uint64)
        g = int(n_u.shape[0])
        if not hasattr(eu, "data_ptr"):
            eu, ev = _host(eu, np.uint32), _host(ev, np.uint32)
            sign = _host(sign, np.uint8 if flags & BBC_SIGNS_2BIT_PACKED else np.int8)
        pe, dev = _ptr(eu)
        pv, _ = _ptr(ev)
        ps, _ = _ptr(sign)
        if dev:
            flags |= BBC_IN_DEVICE_PTRS
        out = (ctypes.c_void_p * g)()
        self._check(lib.bbc_build_csr_batch(self.handle, g, _ptr(n_u)[0], _ptr(n_v)[0], _ptr(off)[0],
                                            pe, pv, ps, flags, out))
        return [Graph(self, out[i]) for i in range(g)]

    # -- counting
    def count_global(self, g: Graph, p: int = 3, q: int = 3) -> int:
        out = ctypes.c_int64()
        self._check(lib.bbc_count_global(self.handle, g.handle, p, q, ctypes.byref(out)))
        return out.value

    def count_bbwc(self, g: Graph, p: int = 3, q: int = 3) -> int:
        """The count by the wedge-centric path (bbc_count_bbwc)."""
        out = ctypes.c_int64(0)
        self._check(lib.bbc_count_bbwc(self.handle, g.handle, p, q, ctypes.byref(out)))
        return out.value

    def top_vertices(self, g: Graph, side: int, k: int) -> Tuple[np.ndarray, np.ndarray]:
        """The k vertices of a side in the most balanced (3,3)-bicliques:
        (ids, counts), counts descending, ties to the smaller id."""
        ids = np.zeros(max(k, 1), dtype=np.uint32)
        cnt = np.zeros(max(k, 1), dtype=np.int64)
        n = _u32(0)
        self._check(lib.bbc_top_vertices(self.handle, g.handle, side, k,
                                         ids.ctypes.data_as(ctypes.c_void_p),
                                         cnt.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return ids[:n.value].copy(), cnt[:n.value].copy()

    def count_through_edges(self, g: Graph, eu, ev, es) -> np.ndarray:
        """Balanced (3,3)-bicliques through each queried edge (eu[i], ev[i])
        taken with sign es[i] (+1 / -1): the change of the count when the edge
        is inserted with that sign (bbc_count_through_edges)."""
        eu = np.ascontiguousarray(eu, dtype=np.uint32)
        ev = np.ascontiguousarray(ev, dtype=np.uint32)
        es = np.ascontiguousarray(es, dtype=np.int8)
        if not (eu.shape == ev.shape == es.shape) or eu.ndim != 1:
            raise ValueError("eu, ev, es must be 1-D arrays of one length")
        out = np.zeros(eu.shape[0], dtype=np.int64)
        self._check(lib.bbc_count_through_edges(self.handle, g.handle, eu.shape[0],
                                                eu.ctypes.data_as(ctypes.c_void_p),
                                                ev.ctypes.data_as(ctypes.c_void_p),
                                                es.ctypes.data_as(ctypes.c_void_p),
                                                out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def count_per_vertex(self, g: Graph, side: int, p: int = 3, q: int = 3, out=None):
        """(per-vertex counts, global count). `out` may be a device tensor of
        int64 (n_u or n_v entries) on the context's device: it is filled on
        the GPU and returned; otherwise a numpy array is returned."""
        info = g.info()
        n = info.n_u if side == 0 else info.n_v
        total = ctypes.c_int64()
        if out is not None:
            if not hasattr(out, "data_ptr") or out.numel() < n or out.element_size() != 8:
                raise ValueError("out must be a tensor of at least n int64 entries")
            self._check(lib.bbc_count_per_vertex(self.handle, g.handle, p, q, side,
                                                 ctypes.c_void_p(out.data_ptr()), ctypes.byref(total)))
            return out, total.value
        arr = np.zeros(max(n, 1), np.int64)
        self._check(lib.bbc_count_per_vertex(self.handle, g.handle, p, q, side,
                                             arr.ctypes.data_as(ctypes.c_void_p), ctypes.byref(total)))
        return arr[:n], total.value

    def count_batch(self, graphs: Sequence[Graph]) -> np.ndarray:
        n = len(graphs)
        hs = (ctypes.c_void_p * max(n, 1))(*[g.handle.value for g in graphs])
        out = np.zeros(max(n, 1), np.int64)
        self._check(lib.bbc_count_batch(self.handle, hs, n, out.ctypes.data_as(ctypes.c_void_p)))
        return out[:n]

    def last_stats(self) -> dict:
        s = CountStats()
        self._check(lib.bbc_get_last_stats(self.handle, ctypes.byref(s)))
        return {k: (float(getattr(s, k)) if k.startswith("ms_") else int(getattr(s, k)))
                for k, _ in CountStats._fields_}

    def set_timing(self, enable: bool = True):
        self._check(lib.bbc_set_timing(self.handle, 1 if enable else 0))

    def memory_stats(self) -> dict:
        m = MemoryStats()
        self._check(lib.bbc_get_memory_stats(self.handle, ctypes.byref(m)))
        return {k: int(getattr(m, k)) for k, _ in MemoryStats._fields_}

    def set_test_hook(self, hook: int, value: int):
        """Host-forced test conditions (BBC_HOOK_*); value 0 resets."""
        self._check(lib.bbc_set_test_hook(self.handle, hook, int(value)))

    # -- serving
    def submit(self, g: Graph) -> int:
        t = ctypes.c_uint64()
        self._check(lib.bbc_submit(self.handle, g.handle, ctypes.byref(t)))
        return t.value

    def submit_coo(self, n_u: int, n_v: int, eu, ev, sign, flags: int = 0) -> int:
        eu, ev = _host(eu, np.uint32), _host(ev, np.uint32)
        sign = _host(sign, np.uint8 if flags & BBC_SIGNS_2BIT_PACKED else np.int8)
        t = ctypes.c_uint64()
        self._check(lib.bbc_submit_coo(self.handle, n_u, n_v, eu.shape[0], _ptr(eu)[0], _ptr(ev)[0],
                                       _ptr(sign)[0], flags, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> Optional[int]:
        out = ctypes.c_int64()
        st = lib.bbc_poll(self.handle, ticket, ctypes.byref(out))
        if st == BBC_E_NOT_READY:
            return None
        self._check(st)
        return out.value

    def wait(self, ticket: int) -> int:
        out = ctypes.c_int64()
        self._check(lib.bbc_wait(self.handle, ticket, ctypes.byref(out)))
        return out.value


def pack_signs_2bit(sign: np.ndarray) -> np.ndarray:
    """+1 / -1 int8 signs -> 2-bit codes (01 = +1, 11 = -1), 4 per byte."""
    s = np.asarray(sign)
    codes = np.where(s < 0, 3, 1).astype(np.uint8)
    pad = (-codes.size) % 4
    codes = np.concatenate([codes, np.zeros(pad, np.uint8)]).reshape(-1, 4)
    return (codes[:, 0] | (codes[:, 1] << 2) | (codes[:, 2] << 4) | (codes[:, 3] << 6)).astype(np.uint8)
