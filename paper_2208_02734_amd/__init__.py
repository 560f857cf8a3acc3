"""Python binding of libmask.so, the MI355X (gfx950) implementation of the
MASK hot path (multilevel approximate similarity search with k-means).

Argument marshalling only: every step of the build and of the query runs in
the library's HIP kernels.  PyTorch provides device memory (tensors, and the
caching allocator the library allocates through) and the current stream.
The functions keep the C names of ``include/mask.h``.  When the library is
not built the import succeeds but every call raises ``MaskError``; there is
no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MASK_LIBRARY") or os.path.join(_HERE, "_lib", "libmask.so")

MASK_OK = 0
_STATUS = {0: "MASK_OK", 1: "MASK_ERR_INVALID", 2: "MASK_ERR_NOMEM", 3: "MASK_ERR_DEVICE",
           4: "MASK_ERR_UNSUPPORTED", 5: "MASK_ERR_BUSY", 6: "MASK_ERR_SHUTDOWN"}
METRICS = {"l2": 0, "l1": 1}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2}
MAX_LEVELS = 16


class MaskError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class mask_matrix(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("n", ctypes.c_int64), ("dim", ctypes.c_int32),
                ("ld", ctypes.c_int32), ("x", ctypes.c_void_p), ("indptr", ctypes.c_void_p),
                ("indices", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("nnz", ctypes.c_int64)]


class mask_level(ctypes.Structure):
    _fields_ = [("n_chunks", ctypes.c_int32), ("k", ctypes.c_int32)]


class mask_build_params(ctypes.Structure):
    _fields_ = [("metric", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("levels", ctypes.POINTER(mask_level)),
                ("lloyd_iters", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("rerank_factor", ctypes.c_int32), ("perm", ctypes.c_void_p),
                ("group_off", ctypes.POINTER(ctypes.c_int64)), ("init", ctypes.c_int32)]


class mask_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("metric", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("level_size", ctypes.c_int64 * MAX_LEVELS), ("device_bytes", ctypes.c_int64),
                ("refined_last_level", ctypes.c_int64), ("layout", ctypes.c_int32),
                ("nnz", ctypes.c_int64)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                            ctypes.c_void_p)


class mask_allocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


class mask_server_params(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_int64), ("max_batch_queries", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("batch_window_us", ctypes.c_int32),
                ("beam_eighths", ctypes.c_int32 * MAX_LEVELS)]


class mask_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted_requests", "submitted_queries", "completed_requests", "completed_queries",
        "batches", "batched_queries", "peak_arena_bytes", "arena_used_bytes",
        "queued_requests", "inflight_batches")]


_lib = None

EXPORTED = ["mask_plan_levels", "mask_build", "mask_query", "mask_query_beams", "mask_query_ragged",
            "mask_query_range", "mask_point_query", "mask_relocate", "mask_insert",
            "mask_kmeanspp", "mask_query_screened", "mask_query_screened_debug",
            "mask_query_screened_noalloc", "mask_query_batched", "mask_query_batched_debug",
            "mask_batched_bytes",
            "mask_query_beams_debug", "mask_screen_bytes",
            "mask_query_debug", "mask_free",
            "mask_index_info", "mask_export_level", "mask_import", "mask_kmeans",
            "mask_last_error", "mask_timing_enable", "mask_timing_report", "mask_clock",
            "mask_server_create", "mask_server_submit", "mask_server_poll",
            "mask_server_stats_get", "mask_server_replay", "mask_server_destroy"]


def lib() -> ctypes.CDLL:
    """The loaded library; raises MaskError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MaskError(3, f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2208_02734_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, VP = ctypes.POINTER, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.mask_plan_levels.argtypes = [I64, I32, I32, P(mask_level), I32, P(I32)]
    L.mask_build.argtypes = [P(mask_matrix), P(mask_build_params), P(mask_allocator), VP, P(VP)]
    L.mask_query.argtypes = [VP, P(mask_matrix), I32, I32, VP, VP, VP]
    L.mask_query_debug.argtypes = [VP, P(mask_matrix), I32, I32, VP, VP, VP, VP]
    L.mask_query_ragged.argtypes = [VP, P(mask_matrix), VP, VP, VP, I32, I32, VP, VP, VP, VP]
    L.mask_query_beams.argtypes = [VP, P(mask_matrix), I32, VP, VP, VP, VP]
    L.mask_query_range.argtypes = [VP, P(mask_matrix), VP, I32, I32, VP, VP, VP, VP]
    L.mask_point_query.argtypes = [VP, P(mask_matrix), VP, VP, VP, VP, VP]
    L.mask_relocate.argtypes = [VP, VP, VP, VP, P(I64), I32, P(I32), P(mask_allocator), VP]
    L.mask_insert.argtypes = [VP, P(mask_matrix), I32, VP, P(I32), P(mask_allocator), VP]
    L.mask_kmeanspp.argtypes = [P(mask_matrix), I32, I32, ctypes.c_uint64, I32, VP, VP,
                                P(mask_allocator), VP]
    L.mask_query_screened.argtypes = [VP, P(mask_matrix), I32, VP, VP, VP, VP, I64, VP]
    L.mask_query_screened_debug.argtypes = [VP, P(mask_matrix), I32, VP, VP, VP, VP, VP, I64,
                                            VP]
    L.mask_query_screened_noalloc.argtypes = [VP, P(mask_matrix), I32, VP, VP, VP, VP]
    L.mask_query_batched.argtypes = [VP, P(mask_matrix), I32, VP, VP, VP, VP, I64, VP]
    L.mask_query_batched_debug.argtypes = [VP, P(mask_matrix), I32, VP, VP, VP, VP, VP, I64, VP]
    L.mask_batched_bytes.argtypes = [VP, VP, I64, P(I64)]
    L.mask_query_beams_debug.argtypes = [VP, P(mask_matrix), I32, VP, VP, VP, VP, VP]
    L.mask_screen_bytes.argtypes = [VP, P(I64)]
    L.mask_free.argtypes = [VP]
    L.mask_index_info.argtypes = [VP, P(mask_info)]
    L.mask_export_level.argtypes = [VP, I32, VP, VP]
    L.mask_import.argtypes = [P(mask_matrix), I32, P(mask_level), P(VP), P(VP),
                              P(mask_build_params), P(mask_allocator), VP, P(VP)]
    L.mask_kmeans.argtypes = [P(mask_matrix), I32, I32, I32, I32, VP, VP, VP, VP,
                              P(mask_allocator), VP]
    L.mask_timing_enable.argtypes = [I32]
    L.mask_timing_report.argtypes = [ctypes.c_char_p, I64, P(I64)]
    L.mask_clock.restype = ctypes.c_double
    L.mask_clock.argtypes = []
    L.mask_server_create.argtypes = [VP, P(mask_server_params), P(mask_allocator), P(VP)]
    L.mask_server_submit.argtypes = [VP, VP, I32, I32, I32, ctypes.c_double,
                                     P(ctypes.c_uint64)]
    L.mask_server_poll.argtypes = [VP, ctypes.c_uint64, P(I32), VP, VP, P(ctypes.c_double)]
    L.mask_server_stats_get.argtypes = [VP, P(mask_server_stats)]
    L.mask_server_destroy.argtypes = [VP]
    L.mask_server_replay.argtypes = [VP, VP, I64, I64, VP, VP, VP, VP, VP, VP,
                                     P(ctypes.c_double)]
    L.mask_last_error.restype = ctypes.c_char_p
    L.mask_last_error.argtypes = []
    for name in EXPORTED:
        if name not in ("mask_last_error", "mask_clock"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != MASK_OK:
        raise MaskError(status, lib().mask_last_error().decode(errors="replace"))


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class CsrTensor:
    """CSR rows on the device: indptr int64[n+1], indices int32[nnz] (strictly
    increasing within a row), values float32[nnz], ``n_cols`` columns."""

    def __init__(self, indptr, indices, values, n_cols: int):
        torch = _torch()
        for t, dt in ((indptr, torch.int64), (indices, torch.int32), (values, torch.float32)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or t.dim() != 1:
                raise MaskError(1, "CSR arrays: CUDA tensors indptr int64, indices int32, "
                                   "values float32")
        self.indptr = indptr.contiguous()
        self.indices = indices.contiguous()
        self.values = values.contiguous()
        self.n_cols = int(n_cols)

    @classmethod
    def from_host(cls, indptr, indices, values, n_cols: int, device="cuda"):
        torch = _torch()
        return cls(torch.from_numpy(np.ascontiguousarray(indptr, dtype=np.int64)).to(device),
                   torch.from_numpy(np.ascontiguousarray(indices, dtype=np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(values, dtype=np.float32)).to(device),
                   n_cols)

    @property
    def shape(self):
        return (self.indptr.shape[0] - 1, self.n_cols)

    @property
    def device(self):
        return self.indptr.device

    def rows(self, lo: int, hi: int) -> "CsrTensor":
        """Rows lo..hi-1 as a new CsrTensor (device copies)."""
        ptr = self.indptr[lo:hi + 1]
        b, e = int(ptr[0].item()), int(ptr[-1].item())
        return CsrTensor((ptr - b).contiguous(), self.indices[b:e].clone(),
                         self.values[b:e].clone(), self.n_cols)


def _matrix(t) -> mask_matrix:
    if isinstance(t, CsrTensor):
        m = mask_matrix()
        m.layout = 1
        m.n = t.shape[0]
        m.dim = t.n_cols
        m.ld = 0
        m.indptr = t.indptr.data_ptr()
        m.indices = t.indices.data_ptr()
        m.values = t.values.data_ptr()
        m.nnz = t.indices.shape[0]
        return m
    return _dense(t)


def _dense(t) -> mask_matrix:
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2:
        raise MaskError(1, "expected a 2-D float32 CUDA tensor")
    if t.shape[0] > 0 and t.stride(1) != 1:
        raise MaskError(1, "rows must be contiguous")
    m = mask_matrix()
    m.layout = 0
    m.n = t.shape[0]
    m.dim = t.shape[1]
    m.ld = t.stride(0) if t.shape[0] > 1 else t.shape[1]
    m.x = t.data_ptr()
    return m


class _TorchAllocator:
    """mask_allocator backed by PyTorch's caching allocator."""

    def __init__(self, device: int):
        torch = _torch()
        self.device = device

        def _alloc(ctx, nbytes, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
            except Exception:  # out of memory -> the library reports MASK_ERR_NOMEM
                return None

        def _free(ctx, ptr, nbytes, stream):
            torch.cuda.caching_allocator_delete(ptr)

        self._a = _ALLOC_FN(_alloc)
        self._f = _FREE_FN(_free)
        self.struct = mask_allocator(None, self._a, self._f)


class Index:
    """Owner of a mask_index handle."""

    def __init__(self, handle: int, allocator=None, metric: str = "l2"):
        self.handle = ctypes.c_void_p(handle)
        self._allocator = allocator  # keeps the callbacks alive as long as the index
        self.metric = metric

    def info(self) -> dict:
        inf = mask_info()
        _check(lib().mask_index_info(self.handle, ctypes.byref(inf)))
        return {"n": inf.n, "dim": inf.dim, "n_levels": inf.n_levels, "metric": inf.metric,
                "precision": inf.precision,
                "level_size": [inf.level_size[i] for i in range(inf.n_levels)],
                "device_bytes": inf.device_bytes,
                "refined_last_level": inf.refined_last_level,
                "layout": "csr" if inf.layout == 1 else "dense", "nnz": inf.nnz}

    def export_level(self, level: int) -> Tuple[np.ndarray, np.ndarray]:
        """(prototypes n_l x dim in chunk-major id order, parent id of each
        item one level down)."""
        inf = self.info()
        n_l = inf["level_size"][level - 1]
        n_below = inf["n"] if level == 1 else inf["level_size"][level - 2]
        P = np.empty((n_l, inf["dim"]), dtype=np.float32)
        par = np.empty(n_below, dtype=np.int32)
        _check(lib().mask_export_level(self.handle, level, P.ctypes.data, par.ctypes.data))
        return P, par

    def free(self):
        if self.handle and self.handle.value:
            lib().mask_free(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _levels_array(levels: Sequence[Tuple[int, int]]):
    arr = (mask_level * len(levels))()
    for i, (c, k) in enumerate(levels):
        arr[i].n_chunks = int(c)
        arr[i].k = int(k)
    return arr


def mask_plan_levels(n: int, length_group: int, n_centroids: int) -> List[Tuple[int, int]]:
    out = (mask_level * (MAX_LEVELS * 4))()
    cnt = ctypes.c_int32()
    _check(lib().mask_plan_levels(n, length_group, n_centroids, out, MAX_LEVELS * 4,
                                  ctypes.byref(cnt)))
    return [(out[i].n_chunks, out[i].k) for i in range(cnt.value)]


INITS = {"first": 0, "kmeans++": 1}


def _params(levels, iters, seed, metric, precision, rerank_factor, perm, group_off=None,
            init="first"):
    lv = _levels_array(levels)
    p = mask_build_params()
    p.metric = METRICS[metric]
    p.precision = PRECISIONS[precision]
    p.n_levels = len(levels)
    p.levels = lv
    p.lloyd_iters = iters
    p.seed = seed & 0xFFFFFFFFFFFFFFFF
    p.rerank_factor = rerank_factor
    p.perm = perm.data_ptr() if perm is not None else None
    p.init = INITS[init]
    if group_off is not None:
        off = np.ascontiguousarray(group_off, dtype=np.int64)
        if off.shape != (levels[0][0] + 1,):
            raise MaskError(1, "group_off must hold levels[0] n_chunks + 1 entries")
        p._group_off = off  # kept alive with the struct
        p.group_off = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    return p, lv


def mask_build(data, levels: Sequence[Tuple[int, int]], iters: int = 30, seed: int = 0,
               metric: str = "l2", precision: str = "fp32", perm=None, rerank_factor: int = 0,
               stream=None, torch_allocator: bool = True, group_off=None,
               init: str = "first") -> Index:
    """Algorithm 1 on a device tensor (n x dim float32) or a CsrTensor;
    returns the index.  perm (int32 CUDA tensor) and group_off (host int64,
    levels[0] n_chunks + 1 entries) give the level-0 order and groups."""
    torch = _torch()
    m = _matrix(data)
    if perm is not None and (perm.dtype != torch.int32 or not perm.is_cuda):
        raise MaskError(1, "perm must be an int32 CUDA tensor")
    p, lv = _params(levels, iters, seed, metric, precision, rerank_factor, perm, group_off,
                    init)
    alloc = _TorchAllocator(data.device.index or 0) if torch_allocator else None
    h = ctypes.c_void_p()
    _check(lib().mask_build(ctypes.byref(m), ctypes.byref(p),
                            ctypes.byref(alloc.struct) if alloc else None,
                            _stream_handle(stream), ctypes.byref(h)))
    return Index(h.value, alloc, metric)


def mask_query(index: Index, queries, k: int, r: int, stream=None, debug: bool = False):
    """Descent for every row of ``queries``; returns (ids int32, dist float32)
    tensors of shape (nq, k), plus the kept prototypes per level when
    ``debug``."""
    torch = _torch()
    m = _matrix(queries)
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    if debug:
        L = index.info()["n_levels"]
        sel = torch.empty((nq, L, r), dtype=torch.int32, device=queries.device)
        _check(lib().mask_query_debug(index.handle, ctypes.byref(m), k, r, ids.data_ptr(),
                                      dist.data_ptr(), sel.data_ptr(), _stream_handle(stream)))
        return ids, dist, sel
    _check(lib().mask_query(index.handle, ctypes.byref(m), k, r, ids.data_ptr(),
                            dist.data_ptr(), _stream_handle(stream)))
    return ids, dist


def mask_query_beams(index: Index, queries, k: int, beams: Sequence[int], stream=None,
                     debug: bool = False):
    """Descent keeping beams[i] prototypes at level i counted from the top;
    returns (ids, dist) like mask_query, plus the kept prototypes per level
    (nq, n_levels, max(beams)) when ``debug``."""
    torch = _torch()
    m = _matrix(queries)
    nq = queries.shape[0]
    b = (ctypes.c_int32 * len(beams))(*[int(x) for x in beams])
    ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    if debug:
        sel = torch.empty((nq, len(beams), max(int(x) for x in beams)), dtype=torch.int32,
                          device=queries.device)
        _check(lib().mask_query_beams_debug(index.handle, ctypes.byref(m), k, b,
                                            ids.data_ptr(), dist.data_ptr(), sel.data_ptr(),
                                            _stream_handle(stream)))
        return ids, dist, sel
    _check(lib().mask_query_beams(index.handle, ctypes.byref(m), k, b, ids.data_ptr(),
                                  dist.data_ptr(), _stream_handle(stream)))
    return ids, dist


def mask_screen_bytes(index: Index) -> int:
    b = ctypes.c_int64()
    _check(lib().mask_screen_bytes(index.handle, ctypes.byref(b)))
    return b.value


def mask_query_screened(index: Index, queries, k: int, beams: Sequence[int], workspace=None,
                        stream=None, debug: bool = False):
    """mask_query_beams with the small prototype levels screened by a BF16
    GEMM (BF16 form); workspace: a CUDA tensor (allocated here for the whole
    batch when None).  Returns (ids, dist) tensors of shape (nq, k), plus the
    kept prototypes per level (nq, n_levels, max(beams)) when ``debug``."""
    torch = _torch()
    m = _matrix(queries)
    nq = queries.shape[0]
    if workspace is None:
        nbytes = max(256, mask_screen_bytes(index) * nq)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=queries.device)
    ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    r = (ctypes.c_int32 * len(beams))(*[int(b) for b in beams])
    ws_bytes = workspace.numel() * workspace.element_size()
    if debug:
        sel = torch.empty((nq, len(beams), max(int(x) for x in beams)), dtype=torch.int32,
                          device=queries.device)
        _check(lib().mask_query_screened_debug(index.handle, ctypes.byref(m), int(k), r,
                                               ids.data_ptr(), dist.data_ptr(), sel.data_ptr(),
                                               workspace.data_ptr(), ws_bytes,
                                               _stream_handle(stream)))
        return ids, dist, sel
    _check(lib().mask_query_screened(index.handle, ctypes.byref(m), int(k), r, ids.data_ptr(),
                                     dist.data_ptr(), workspace.data_ptr(), ws_bytes,
                                     _stream_handle(stream)))
    return ids, dist


def mask_batched_bytes(index: Index, beams: Sequence[int], n_queries: int) -> int:
    """Workspace bytes of mask_query_batched for one slice of n_queries."""
    b = ctypes.c_int64()
    r = (ctypes.c_int32 * len(beams))(*[int(x) for x in beams])
    _check(lib().mask_batched_bytes(index.handle, r, int(n_queries), ctypes.byref(b)))
    return b.value


def mask_query_batched(index: Index, queries, k: int, beams: Sequence[int], workspace=None,
                       stream=None, debug: bool = False):
    """mask_query_screened with the data layer evaluated leaf by leaf (BF16
    form, dim <= 256); the same results.  workspace: a CUDA tensor
    (allocated here for the whole batch, or 2^20 queries, when None).
    Returns (ids, dist), plus the kept prototypes per level when ``debug``."""
    torch = _torch()
    m = _matrix(queries)
    nq = queries.shape[0]
    if workspace is None:
        nbytes = mask_batched_bytes(index, beams, max(1, min(nq, 1 << 20)))
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=queries.device)
    ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    r = (ctypes.c_int32 * len(beams))(*[int(b) for b in beams])
    ws_bytes = workspace.numel() * workspace.element_size()
    if debug:
        sel = torch.empty((nq, len(beams), max(int(x) for x in beams)), dtype=torch.int32,
                          device=queries.device)
        _check(lib().mask_query_batched_debug(index.handle, ctypes.byref(m), int(k), r,
                                              ids.data_ptr(), dist.data_ptr(), sel.data_ptr(),
                                              workspace.data_ptr(), ws_bytes,
                                              _stream_handle(stream)))
        return ids, dist, sel
    _check(lib().mask_query_batched(index.handle, ctypes.byref(m), int(k), r, ids.data_ptr(),
                                    dist.data_ptr(), workspace.data_ptr(), ws_bytes,
                                    _stream_handle(stream)))
    return ids, dist


def mask_query_screened_noalloc(index: Index, queries, k: int, beams: Sequence[int],
                                stream=None, out=None):
    """mask_query_screened on the library's static per-GPU scratch: no
    workspace.  ``out``: optional (ids, dist) tensors of shape (nq, k) to
    write into (allocated here when None).  Returns (ids, dist)."""
    torch = _torch()
    m = _matrix(queries)
    nq = queries.shape[0]
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    else:
        ids, dist = out
    r = (ctypes.c_int32 * len(beams))(*[int(b) for b in beams])
    _check(lib().mask_query_screened_noalloc(index.handle, ctypes.byref(m), int(k), r,
                                             ids.data_ptr(), dist.data_ptr(),
                                             _stream_handle(stream)))
    return ids, dist


def mask_query_ragged(index: Index, queries, k_i, r_i, stream=None, k_max: int = 0,
                      r_max: int = 0, beam_eighths: Optional[Sequence[int]] = None):
    """Per-query k and r (int32 CUDA tensors of length nq); returns
    (ids, dist, offsets): query i's results are ids[offsets[i]:offsets[i+1]].
    k_max / r_max: bounds passed to the library (raised to the largest k_i /
    r_i when smaller).  beam_eighths: optional beam profile (one entry per
    level, top first): query i keeps ceil(r_i * e / 8) prototypes there."""
    torch = _torch()
    m = _matrix(queries)
    k_i = k_i.to(device=queries.device, dtype=torch.int32).contiguous()
    r_i = r_i.to(device=queries.device, dtype=torch.int32).contiguous()
    off = torch.zeros(queries.shape[0] + 1, dtype=torch.int64, device=queries.device)
    off[1:] = torch.cumsum(k_i.to(torch.int64), 0)
    total = int(off[-1].item())
    ids = torch.empty(max(total, 1), dtype=torch.int32, device=queries.device)
    dist = torch.empty(max(total, 1), dtype=torch.float32, device=queries.device)
    k_max = max(int(k_max), int(k_i.max().item()) if queries.shape[0] else 1)
    r_max = max(int(r_max), int(r_i.max().item()) if queries.shape[0] else 1)
    prof = None
    if beam_eighths is not None:
        prof = (ctypes.c_int32 * len(beam_eighths))(*[int(e) for e in beam_eighths])
    _check(lib().mask_query_ragged(index.handle, ctypes.byref(m), k_i.data_ptr(), r_i.data_ptr(),
                                   off.data_ptr(), k_max, r_max, prof, ids.data_ptr(),
                                   dist.data_ptr(), _stream_handle(stream)))
    return ids[:total], dist[:total], off


def mask_query_range(index: Index, queries, radius, max_out: int, level_cap: int, stream=None):
    """Range search (Algorithm 3); radius: a float or a float32 CUDA tensor
    of length nq.  Returns (ids (nq x max_out), dist, count) tensors."""
    torch = _torch()
    m = _matrix(queries)
    nq = queries.shape[0]
    if not isinstance(radius, torch.Tensor):
        radius = torch.full((nq,), float(radius), dtype=torch.float32, device=queries.device)
    radius = radius.to(device=queries.device, dtype=torch.float32).contiguous()
    ids = torch.empty((nq, max_out), dtype=torch.int32, device=queries.device)
    dist = torch.empty((nq, max_out), dtype=torch.float32, device=queries.device)
    count = torch.empty(nq, dtype=torch.int32, device=queries.device)
    _check(lib().mask_query_range(index.handle, ctypes.byref(m), radius.data_ptr(), int(max_out),
                                  int(level_cap), ids.data_ptr(), dist.data_ptr(),
                                  count.data_ptr(), _stream_handle(stream)))
    return ids, dist, count


def mask_point_query(index: Index, queries, stream=None):
    """Point query (Section 3.3) for every row of ``queries``; returns
    (ids, dist, leaf, match) tensors of length nq."""
    torch = _torch()
    m = _matrix(queries)
    nq = queries.shape[0]
    dev = queries.device
    ids = torch.empty(nq, dtype=torch.int32, device=dev)
    dist = torch.empty(nq, dtype=torch.float32, device=dev)
    leaf = torch.empty(nq, dtype=torch.int32, device=dev)
    match = torch.empty(nq, dtype=torch.int32, device=dev)
    _check(lib().mask_point_query(index.handle, ctypes.byref(m), ids.data_ptr(),
                                  dist.data_ptr(), leaf.data_ptr(), match.data_ptr(),
                                  _stream_handle(stream)))
    return ids, dist, leaf, match


def mask_relocate(index: Index, leaf, wrong, stream=None):
    """One relocation step; leaf and wrong are int32 CUDA tensors of length
    n in data row order.  Returns (perm int32 CUDA tensor, group_off numpy
    int64) for the rebuild."""
    torch = _torch()
    info = index.info()
    n = info["n"]
    if leaf.dtype != torch.int32 or wrong.dtype != torch.int32 or leaf.numel() != n \
            or wrong.numel() != n:
        raise MaskError(1, "leaf and wrong must be int32 tensors of length n")
    leaf, wrong = leaf.contiguous(), wrong.contiguous()
    perm = torch.empty(n, dtype=torch.int32, device=leaf.device)
    cap = n + 1
    off = np.zeros(cap, dtype=np.int64)
    ng = ctypes.c_int32()
    alloc = _TorchAllocator(leaf.device.index or 0)
    _check(lib().mask_relocate(index.handle, leaf.data_ptr(), wrong.data_ptr(), perm.data_ptr(),
                               off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cap,
                               ctypes.byref(ng), ctypes.byref(alloc.struct),
                               _stream_handle(stream)))
    return perm, off[:ng.value + 1].copy()


def mask_insert(index: Index, points, max_leaf: int = 0, stream=None):
    """Dynamic insertion of the rows of ``points`` (float32 CUDA tensor);
    returns (leaf of every new row, number of groups rebuilt).  The new rows
    take the next ids."""
    torch = _torch()
    m = _matrix(points)
    leaf = torch.empty(points.shape[0], dtype=torch.int32, device=points.device)
    nr = ctypes.c_int32()
    alloc = _TorchAllocator(points.device.index or 0)
    _check(lib().mask_insert(index.handle, ctypes.byref(m), int(max_leaf), leaf.data_ptr(),
                             ctypes.byref(nr), ctypes.byref(alloc.struct),
                             _stream_handle(stream)))
    return leaf, nr.value


def mask_free(index: Index):
    index.free()


def mask_import(data, levels: Sequence[Tuple[int, int]], protos: Sequence[np.ndarray],
                parents: Sequence[np.ndarray], metric: str = "l2", precision: str = "fp32",
                rerank_factor: int = 0, stream=None, torch_allocator: bool = True) -> Index:
    """Index from prototypes (chunk-major, per level) and parent ids (per
    level, for the items one level down), e.g. built by another
    implementation."""
    m = _matrix(data)
    L = len(levels)
    P = [np.ascontiguousarray(p, dtype=np.float32) for p in protos]
    Q = [np.ascontiguousarray(q, dtype=np.int32) for q in parents]
    pp = (ctypes.c_void_p * L)(*[p.ctypes.data for p in P])
    qq = (ctypes.c_void_p * L)(*[q.ctypes.data for q in Q])
    prm, lv = _params(levels, 0, 0, metric, precision, rerank_factor, None)
    alloc = _TorchAllocator(data.device.index or 0) if torch_allocator else None
    h = ctypes.c_void_p()
    _check(lib().mask_import(ctypes.byref(m), L, _levels_array(levels), pp, qq,
                             ctypes.byref(prm), ctypes.byref(alloc.struct) if alloc else None,
                             _stream_handle(stream), ctypes.byref(h)))
    return Index(h.value, alloc, metric)


def mask_kmeanspp(items, n_chunks: int, k: int, seed: int, level: int = 1, stream=None):
    """k-means++ seeds of every group of a device tensor; returns
    (centroids (n_chunks*k x dim), chosen item indices int32)."""
    torch = _torch()
    m = _matrix(items)
    np_ = n_chunks * k
    cent = torch.empty((np_, items.shape[1]), dtype=torch.float32, device=items.device)
    chosen = torch.empty(np_, dtype=torch.int32, device=items.device)
    alloc = _TorchAllocator(items.device.index or 0)
    _check(lib().mask_kmeanspp(ctypes.byref(m), int(n_chunks), int(k),
                               ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), int(level),
                               cent.data_ptr(), chosen.data_ptr(), ctypes.byref(alloc.struct),
                               _stream_handle(stream)))
    return cent, chosen


def mask_kmeans(items, n_chunks: int, k: int, iters: int, init=None, metric: str = "l2",
                stream=None):
    """Batched per-group Lloyd on a device tensor or CsrTensor; returns (centroids
    (n_chunks*k x dim), labels int32, inertia float64 (iters x n_chunks))."""
    torch = _torch()
    m = _matrix(items)
    dim = items.shape[1]
    cent = torch.empty((n_chunks * k, dim), dtype=torch.float32, device=items.device)
    labels = torch.empty(items.shape[0], dtype=torch.int32, device=items.device)
    inertia = torch.zeros((max(iters, 1), n_chunks), dtype=torch.float64, device=items.device)
    if init is not None:
        init = init.contiguous()
    alloc = _TorchAllocator(items.device.index or 0)
    _check(lib().mask_kmeans(ctypes.byref(m), n_chunks, k, iters, METRICS[metric],
                             init.data_ptr() if init is not None else None, cent.data_ptr(),
                             labels.data_ptr(), inertia.data_ptr(),
                             ctypes.byref(alloc.struct), _stream_handle(stream)))
    return cent, labels, inertia[:iters]


def mask_timing_enable(on: bool = True):
    _check(lib().mask_timing_enable(1 if on else 0))


def mask_timing_report() -> dict:
    """{kernel name: (launches, total milliseconds)} of the instrumented
    launches since timing was enabled; "descent_rows" counts the candidate
    rows the descent evaluated; "kmeanspp_level<l>" times the k-means++
    seeding of level l, and "seeding_rows_read_level<l>" and
    "seeding_rows_lowered_level<l>" count the rows its updates read (not
    ruled out by the triangle inequality) and those whose D^2 fell."""
    need = ctypes.c_int64()
    _check(lib().mask_timing_report(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(int(need.value) + 1)
    _check(lib().mask_timing_report(buf, len(buf), ctypes.byref(need)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def mask_clock() -> float:
    """Seconds on the server's steady clock."""
    return lib().mask_clock()


class MaskServer:
    """Continuous-batching request loop on a resident index (host queries in,
    host results out)."""

    def __init__(self, index: Index, arena_bytes: int = 1 << 30, max_batch_queries: int = 65536,
                 n_streams: int = 2, batch_window_us: int = 0,
                 beam_eighths: Optional[Sequence[int]] = None):
        prof = [int(e) for e in (beam_eighths or [])]
        if len(prof) > MAX_LEVELS:
            raise MaskError(1, "beam profile longer than the level limit")
        p = mask_server_params(int(arena_bytes), int(max_batch_queries), int(n_streams),
                               int(batch_window_us),
                               (ctypes.c_int32 * MAX_LEVELS)(*(prof + [0] * (MAX_LEVELS - len(prof)))))
        h = ctypes.c_void_p()
        _check(lib().mask_server_create(index.handle, ctypes.byref(p), None, ctypes.byref(h)))
        self.handle = h
        self.index = index
        self.dim = index.info()["dim"]
        self._pending = {}

    def submit(self, queries: np.ndarray, k: int, r: int, t_arrival: Optional[float] = None) -> int:
        q = np.ascontiguousarray(queries, dtype=np.float32)
        if q.ndim != 2 or q.shape[1] != self.dim:
            raise MaskError(1, "queries must be n x dim float32")
        t = mask_clock() if t_arrival is None else float(t_arrival)
        ticket = ctypes.c_uint64()
        _check(lib().mask_server_submit(self.handle, q.ctypes.data, q.shape[0], int(k), int(r), t,
                                        ctypes.byref(ticket)))
        self._pending[ticket.value] = (q.shape[0], int(k))
        return ticket.value

    def poll(self, ticket: int):
        """None while running; (ids (n x k), dist (n x k), t_done) when done."""
        n, k = self._pending[ticket]
        ids = np.empty((n, k), dtype=np.int32)
        dist = np.empty((n, k), dtype=np.float32)
        done = ctypes.c_int32()
        t = ctypes.c_double()
        _check(lib().mask_server_poll(self.handle, ticket, ctypes.byref(done), ids.ctypes.data,
                                      dist.ctypes.data, ctypes.byref(t)))
        if not done.value:
            return None
        del self._pending[ticket]
        return ids, dist, t.value

    def stats(self) -> dict:
        st = mask_server_stats()
        _check(lib().mask_server_stats_get(self.handle, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in mask_server_stats._fields_}

    def replay(self, pool: np.ndarray, t_offset, n_q, pool_off, k, r):
        """Open-loop replay of a request schedule from a native thread (see
        mask_server_replay); returns (latency seconds per request, span)."""
        pool = np.ascontiguousarray(pool, dtype=np.float32)
        t = np.ascontiguousarray(t_offset, dtype=np.float64)
        nq = np.ascontiguousarray(n_q, dtype=np.int32)
        off = np.ascontiguousarray(pool_off, dtype=np.int64)
        kk = np.ascontiguousarray(k, dtype=np.int32)
        rr = np.ascontiguousarray(r, dtype=np.int32)
        lat = np.zeros(t.shape[0], dtype=np.float64)
        span = ctypes.c_double()
        _check(lib().mask_server_replay(self.handle, pool.ctypes.data, pool.shape[0], t.shape[0],
                                        t.ctypes.data, nq.ctypes.data, off.ctypes.data,
                                        kk.ctypes.data, rr.ctypes.data, lat.ctypes.data,
                                        ctypes.byref(span)))
        return lat, span.value

    def close(self):
        if self.handle and self.handle.value:
            lib().mask_server_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
