"""ctypes binding of libmessi.so (include/messi.h).

Argument marshalling only: every step of the index build and the search runs
in the library's HIP kernels.  Device memory and streams come from torch.
Loading fails loudly if the library has not been built; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmessi.so")

MESSI_OK = 0
MESSI_EINVAL = -1
MESSI_ENOMEM = -2
MESSI_EDEVICE = -3
MESSI_ENODEV = -4
MESSI_EBUSY = -5
MESSI_EOVERFLOW = -6
MODE_FP32 = 0
MODE_BF16 = 1
MODE_APPROX = 2  # approximate: the best leaf's members only (not exact)
SERVER_BATCH_ONLY = 0x100  # OR into a server mode: launches of one query also use the matrix-core filter
SERVER_NO_GRAPHS = 0x200   # OR into a server mode: eager launches, no HIP graphs
SERVER_SLOTS = 0x400       # OR into a BF16 server mode: the slot engine instead of lanes of batches
MAX_K = 1024

EXPORTED = [
    "messi_build", "messi_build_ex", "messi_knn", "messi_knn_ex", "messi_free", "messi_index_info",
    "messi_export_words", "messi_export_leaves", "messi_znorm", "messi_windows", "messi_knn_dtw", "messi_append",
    "messi_breakpoints", "messi_knn_noalloc",
    "messi_last_error",
    "messi_server_create", "messi_server_submit", "messi_server_poll", "messi_server_stats", "messi_server_clock_ms",
    "messi_server_destroy",
]


class MessiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("messi error %d: %s" % (code, msg))
        self.code = code


class Leaf(ctypes.Structure):
    _fields_ = [("card", ctypes.c_uint8 * 16), ("prefix", ctypes.c_uint8 * 16),
                ("start", ctypes.c_uint32), ("count", ctypes.c_uint32)]


LEAF_DTYPE = np.dtype([("card", np.uint8, (16,)), ("prefix", np.uint8, (16,)),
                       ("start", np.uint32), ("count", np.uint32)])


class Opts(ctypes.Structure):
    _fields_ = [("znorm", ctypes.c_int32), ("bf16_shadow", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("mode", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64),
                ("scan_chunk", ctypes.c_int32), ("cand_cap", ctypes.c_uint32), ("row_filter_max_q", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("len", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("card_bits", ctypes.c_int32), ("leaf_cap", ctypes.c_int32), ("n_leaves", ctypes.c_int64),
                ("max_leaf", ctypes.c_int64), ("levels", ctypes.c_int32), ("has_bf16", ctypes.c_int32),
                ("device_bytes", ctypes.c_uint64), ("data_absmax", ctypes.c_float),
                ("ms_znorm", ctypes.c_double), ("ms_summarize", ctypes.c_double), ("ms_bucket", ctypes.c_double),
                ("ms_split", ctypes.c_double), ("ms_finalize", ctypes.c_double), ("ms_shadow", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("fine_segments", ctypes.c_int32), ("fine_length", ctypes.c_int32)]


class KnnStats(ctypes.Structure):
    _fields_ = [("leaves_total", ctypes.c_int64), ("leaves_kept", ctypes.c_int64),
                ("leaves_scanned", ctypes.c_int64), ("series_bounded", ctypes.c_int64),
                ("series_distance", ctypes.c_int64), ("series_abandoned", ctypes.c_int64),
                ("series_recheck", ctypes.c_int64), ("candidates", ctypes.c_int64), ("bytes_scan", ctypes.c_int64),
                ("ms_total", ctypes.c_double), ("ms_prep", ctypes.c_double), ("ms_leaf_lb", ctypes.c_double),
                ("ms_approx", ctypes.c_double), ("ms_order", ctypes.c_double), ("ms_scan", ctypes.c_double),
                ("ms_final", ctypes.c_double), ("scan_launches", ctypes.c_int32),
                ("scan_ms_control", ctypes.c_double), ("scan_ms_filter", ctypes.c_double),
                ("scan_ms_distance", ctypes.c_double), ("scan_ms_block_mean", ctypes.c_double),
                ("scan_ms_block_max", ctypes.c_double), ("ms_bf16_filter", ctypes.c_double),
                ("ms_bf16_recheck", ctypes.c_double), ("bf16_flops", ctypes.c_int64), ("bf16_rounds", ctypes.c_int32),
                ("reruns", ctypes.c_int32), ("fallbacks", ctypes.c_int32), ("ms_fixup", ctypes.c_double),
                ("bf16_stage_queries", ctypes.c_int32), ("bf16_max_leaf_queries", ctypes.c_int32),
                ("series_word_bounded", ctypes.c_int64), ("series_fine_bounded", ctypes.c_int64),
                ("ms_scan_coarse", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("bf16_batches", ctypes.c_int64), ("row_filter", ctypes.c_int64),
                ("requeued", ctypes.c_int64), ("eager_launches", ctypes.c_int64),
                ("graphs_recorded", ctypes.c_int64), ("graph_replays", ctypes.c_int64),
                ("lanes", ctypes.c_int32), ("batch", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("slot_steps", ctypes.c_int64), ("slot_admitted", ctypes.c_int64), ("slots", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("k", ctypes.c_int32), ("status", ctypes.c_int32),
                ("t_submit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double),
                ("idx", ctypes.c_int64 * MAX_K), ("dist", ctypes.c_float * MAX_K)]


_lib = None


def load():
    """Load libmessi.so; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmessi.so is not built: run python -m paper_2009_00786_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.messi_build.argtypes = [vp, i64, i32, i32, i32, i32]
        lib.messi_build.restype = vp
        lib.messi_build_ex.argtypes = [vp, i64, i32, i32, i32, i32, ctypes.POINTER(Opts)]
        lib.messi_build_ex.restype = vp
        lib.messi_knn.argtypes = [vp, vp, i32, i32, vp, vp]
        lib.messi_knn.restype = ctypes.c_int
        lib.messi_knn_ex.argtypes = [vp, vp, i32, vp, i32, i32, vp, vp, vp, ctypes.POINTER(KnnStats)]
        lib.messi_knn_ex.restype = ctypes.c_int
        lib.messi_knn_noalloc.argtypes = [vp, vp, i32, i32, vp, vp, vp]
        lib.messi_knn_noalloc.restype = ctypes.c_int
        lib.messi_free.argtypes = [vp]
        lib.messi_free.restype = None
        lib.messi_index_info.argtypes = [vp, ctypes.POINTER(Info)]
        lib.messi_index_info.restype = ctypes.c_int
        lib.messi_export_words.argtypes = [vp, vp]
        lib.messi_export_words.restype = ctypes.c_int
        lib.messi_export_leaves.argtypes = [vp, vp, vp]
        lib.messi_export_leaves.restype = ctypes.c_int
        lib.messi_znorm.argtypes = [vp, i64, i32, vp]
        lib.messi_znorm.restype = ctypes.c_int
        lib.messi_windows.argtypes = [vp, i64, i32, i64, i32, vp, vp]
        lib.messi_windows.restype = ctypes.c_int
        lib.messi_knn_dtw.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, ctypes.POINTER(KnnStats)]
        lib.messi_knn_dtw.restype = ctypes.c_int
        lib.messi_append.argtypes = [vp, vp, i64, vp]
        lib.messi_append.restype = ctypes.c_int
        lib.messi_breakpoints.argtypes = [i32, vp]
        lib.messi_breakpoints.restype = ctypes.c_int
        lib.messi_last_error.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        lib.messi_last_error.restype = ctypes.c_int
        lib.messi_server_create.argtypes = [vp, ctypes.c_size_t, i32, i32]
        lib.messi_server_create.restype = vp
        lib.messi_server_submit.argtypes = [vp, vp, i32, ctypes.c_uint64]
        lib.messi_server_submit.restype = ctypes.c_int
        lib.messi_server_poll.argtypes = [vp, ctypes.POINTER(Result), i32]
        lib.messi_server_poll.restype = ctypes.c_int
        lib.messi_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        lib.messi_server_stats.restype = ctypes.c_int
        lib.messi_server_clock_ms.argtypes = [vp]
        lib.messi_server_clock_ms.restype = ctypes.c_double
        lib.messi_server_destroy.argtypes = [vp]
        lib.messi_server_destroy.restype = None
        _lib = lib
    return _lib


def last_error():
    buf = ctypes.create_string_buffer(512)
    code = load().messi_last_error(buf, 512)
    return code, buf.value.decode(errors="replace")


def _check(rc):
    if rc != MESSI_OK:
        code, msg = last_error()
        raise MessiError(rc, msg)


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream)


def breakpoints(card_bits: int) -> np.ndarray:
    out = np.zeros(255, dtype=np.float32)
    _check(load().messi_breakpoints(card_bits, out.ctypes.data))
    return out[:(1 << card_bits) - 1].copy()


def windows(long_series, length, step=1, znorm=True, out=None, stream=None):
    """The windows of a 1-D CUDA fp32 tensor as a [count, length] collection:
    row r is long_series[r * step : r * step + length], z-normalised per
    window when znorm (count = (m - length) // step + 1)."""
    assert long_series.is_cuda and long_series.dtype.is_floating_point and long_series.is_contiguous()
    import torch
    m = long_series.numel()
    if m < length:
        raise MessiError(MESSI_EINVAL, "the long series is shorter than one window")
    count = (m - length) // step + 1 if step >= 1 else 0
    if out is None:
        out = torch.empty((max(count, 1), length), dtype=torch.float32, device=long_series.device)
    _check(load().messi_windows(ctypes.c_void_p(long_series.data_ptr()), m, length, step, int(znorm),
                                ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def znorm_(series, stream=None):
    """z-normalise a CUDA fp32 tensor [n, len] in place (fp64 statistics)."""
    assert series.is_cuda and series.dtype.is_floating_point and series.is_contiguous()
    n, length = series.shape
    _check(load().messi_znorm(ctypes.c_void_p(series.data_ptr()), n, length, _stream_ptr(stream)))
    return series


class Index:
    """An iSAX index over a CUDA fp32 tensor [n, len]; the tensor is borrowed."""

    def __init__(self, series, segments=16, card_bits=8, leaf_cap=2000, znorm=False, bf16_shadow=False,
                 stream=None, mode=MODE_FP32, max_slots=0, budget_bytes=0, scan_chunk=0, cand_cap=0,
                 row_filter_max_q=0):
        """Options as messi_opts (include/messi.h); zeros take the defaults."""
        lib = load()
        if series.is_cuda:
            assert series.is_contiguous()
            n, length = series.shape
            ptr = series.data_ptr()
        else:
            n, length, ptr = 0, 0, 0
        opts = Opts(int(bool(znorm)), int(bool(bf16_shadow)), _stream_ptr(stream), int(mode), int(max_slots),
                    int(budget_bytes), int(scan_chunk), int(cand_cap), int(row_filter_max_q))
        h = lib.messi_build_ex(ctypes.c_void_p(ptr) if ptr else None, n if series.is_cuda else series.shape[0],
                               length if series.is_cuda else series.shape[1], segments, card_bits, leaf_cap,
                               ctypes.byref(opts))
        if not h:
            code, msg = last_error()
            raise MessiError(code, msg)
        self._h = ctypes.c_void_p(h)
        self.series = series  # keep the borrowed tensor alive
        self.segments = segments
        self.card_bits = card_bits
        self.leaf_cap = leaf_cap

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load().messi_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def append(self, series, stream=None):
        """Append rows: `series` is a CUDA tensor [new_n, len] whose first n
        rows are the indexed ones; the index then borrows it."""
        assert series.is_cuda and series.is_contiguous() and series.dim() == 2
        _check(load().messi_append(self._h, ctypes.c_void_p(series.data_ptr()), series.shape[0],
                                   _stream_ptr(stream)))
        self.series = series

    def info(self) -> dict:
        inf = Info()
        _check(load().messi_index_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in Info._fields_}

    def export_words(self) -> np.ndarray:
        n = self.series.shape[0]
        out = np.zeros((n, self.segments), dtype=np.uint8)
        _check(load().messi_export_words(self._h, out.ctypes.data))
        return out

    def export_leaves(self):
        inf = self.info()
        leaves = np.zeros(inf["n_leaves"], dtype=LEAF_DTYPE)
        pos = np.zeros(inf["n"], dtype=np.uint32)
        _check(load().messi_export_leaves(self._h, leaves.ctypes.data, pos.ctypes.data))
        return leaves, pos

    def knn(self, queries, k: int, mode: int = MODE_FP32, stream=None, stats: bool = False, out=None,
            k_per_query=None):
        """Exact k-NN of CUDA fp32 queries [nq, len] -> (idx int64 [nq, k], dist fp32 [nq, k]) on the GPU
        (messi_knn_ex).  k_per_query: optional CUDA int32 [nq] of per-query k <= k; row q then holds
        its k_per_query[q] answers followed by (-1, +inf)."""
        import torch
        assert queries.is_cuda and queries.dtype == torch.float32 and queries.is_contiguous()
        nq = queries.shape[0]
        if out is None:
            out_idx = torch.empty((nq, k), dtype=torch.int64, device=queries.device)
            out_dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
        else:
            out_idx, out_dist = out
        kq = None
        if k_per_query is not None:
            assert k_per_query.is_cuda and k_per_query.dtype == torch.int32 and k_per_query.is_contiguous()
            kq = ctypes.c_void_p(k_per_query.data_ptr())
        st = KnnStats() if stats else None
        rc = load().messi_knn_ex(self._h, ctypes.c_void_p(queries.data_ptr()), nq, kq, k, mode, _stream_ptr(stream),
                                 ctypes.c_void_p(out_idx.data_ptr()), ctypes.c_void_p(out_dist.data_ptr()),
                                 ctypes.byref(st) if st is not None else None)
        _check(rc)
        if stats:
            return out_idx, out_dist, {f: getattr(st, f) for f, _ in KnnStats._fields_}
        return out_idx, out_dist

    def knn_plain(self, queries, k: int):
        """messi_knn: the synchronous plain call (the index's search mode, null stream)."""
        import torch
        assert queries.is_cuda and queries.dtype == torch.float32 and queries.is_contiguous()
        nq = queries.shape[0]
        out_idx = torch.empty((nq, k), dtype=torch.int64, device=queries.device)
        out_dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
        _check(load().messi_knn(self._h, ctypes.c_void_p(queries.data_ptr()), nq, k,
                                ctypes.c_void_p(out_idx.data_ptr()), ctypes.c_void_p(out_dist.data_ptr())))
        return out_idx, out_dist

    def knn_noalloc(self, queries, k: int, out, stream=None):
        """messi_knn_noalloc: the FP32 exact search with its buffers in the library's
        static device array.  `out` = (idx int64 [nq, k], dist fp32 [nq, k]), CUDA,
        caller-allocated (the call itself allocates nothing)."""
        import torch
        assert queries.is_cuda and queries.dtype == torch.float32 and queries.is_contiguous()
        out_idx, out_dist = out
        _check(load().messi_knn_noalloc(self._h, ctypes.c_void_p(queries.data_ptr()), queries.shape[0], k,
                                        _stream_ptr(stream), ctypes.c_void_p(out_idx.data_ptr()),
                                        ctypes.c_void_p(out_dist.data_ptr())))
        return out_idx, out_dist

    def knn_dtw(self, queries, k: int, band: int, stream=None, stats: bool = False, out=None):
        """Exact k-NN under DTW with a Sakoe-Chiba band of half-width `band`
        (the paper's window of 10% of the length is band = len // 10)."""
        import torch
        assert queries.is_cuda and queries.dtype == torch.float32 and queries.is_contiguous()
        nq = queries.shape[0]
        if out is None:
            out_idx = torch.empty((nq, k), dtype=torch.int64, device=queries.device)
            out_dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
        else:
            out_idx, out_dist = out
        st = KnnStats() if stats else None
        rc = load().messi_knn_dtw(self._h, ctypes.c_void_p(queries.data_ptr()), nq, k, band, _stream_ptr(stream),
                                  ctypes.c_void_p(out_idx.data_ptr()), ctypes.c_void_p(out_dist.data_ptr()),
                                  ctypes.byref(st) if st is not None else None)
        _check(rc)
        if stats:
            return out_idx, out_dist, {f: getattr(st, f) for f, _ in KnnStats._fields_}
        return out_idx, out_dist


class Server:
    """Continuous-batching request loop over a resident index (messi_server_*)."""

    def __init__(self, index: Index, budget_bytes: int = 0, max_slots: int = 0, mode: int = MODE_BF16):
        """budget_bytes / max_slots 0: the index's options (messi_server_create)."""
        h = load().messi_server_create(index.handle, budget_bytes, max_slots, mode)
        if not h:
            code, msg = last_error()
            raise MessiError(code, msg)
        self._h = ctypes.c_void_p(h)
        self.index = index
        self._buf = (Result * 64)()

    def submit(self, query: np.ndarray, k: int, tag: int):
        q = np.ascontiguousarray(query, dtype=np.float32)
        rc = load().messi_server_submit(self._h, q.ctypes.data, k, tag)
        _check(rc)

    def poll(self):
        n = load().messi_server_poll(self._h, self._buf, len(self._buf))
        if n < 0:
            _check(n)
        out = []
        for i in range(n):
            r = self._buf[i]
            out.append({"tag": r.tag, "k": r.k, "status": r.status, "t_submit_ms": r.t_submit_ms,
                        "t_done_ms": r.t_done_ms, "idx": np.ctypeslib.as_array(r.idx)[:r.k].copy(),
                        "dist": np.ctypeslib.as_array(r.dist)[:r.k].copy()})
        return out

    def clock_ms(self) -> float:
        return load().messi_server_clock_ms(self._h)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().messi_server_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().messi_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
