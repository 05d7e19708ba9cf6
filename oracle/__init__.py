"""CPU oracle for the MESSI hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2009_00786_amd``) and never imports it.  The arithmetic lives in
``oracle.c`` (plain C, built with gcc -O2 -ffp-contract=off); this module only
marshals numpy arrays.

Each function cites the passage of the paper (Peng, Fatourou, Palpanas,
"MESSI: In-Memory Data Series Indexing") or the textbook definition it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

LEAF_DTYPE = np.dtype([("card", np.uint8, (16,)), ("prefix", np.uint8, (16,)),
                       ("start", np.uint32), ("count", np.uint32)])

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no multiply-add contraction, no fast math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-pthread", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=False)
        lib = ctypes.CDLL(LIB)
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_breakpoints.argtypes = [ctypes.c_int, vp]
        lib.oracle_breakpoints.restype = ctypes.c_int
        lib.oracle_znorm.argtypes = [vp, i64, i32, vp]
        lib.oracle_paa.argtypes = [vp, i64, i32, i32, vp]
        lib.oracle_symbols.argtypes = [vp, i64, i32, i32, vp, vp]
        lib.oracle_root_keys.argtypes = [vp, i64, i32, i32, vp]
        lib.oracle_build_leaves.argtypes = [vp, i64, i32, i32, i64, vp, vp]
        lib.oracle_build_leaves.restype = i64
        lib.oracle_d64.argtypes = [vp, vp, i32]
        lib.oracle_d64.restype = d
        lib.oracle_mindist_sq.argtypes = [vp, i32, i32, vp, vp, i32, vp, d]
        lib.oracle_mindist_sq.restype = d
        lib.oracle_mindist_sq_f.argtypes = [vp, i32, i32, vp, vp, i32, vp]
        lib.oracle_mindist_sq_f.restype = d
        lib.oracle_knn_brute.argtypes = [vp, i64, i32, vp, i32, i32, ctypes.c_int, i64, vp, vp]
        lib.oracle_knn_brute.restype = ctypes.c_int
        lib.oracle_knn_isax.argtypes = [vp, i64, i32, vp, i32, i32, vp, i64, vp, vp, i32, i32, vp, vp, vp]
        lib.oracle_knn_isax.restype = ctypes.c_int
        lib.oracle_build_leaves_ex.argtypes = [vp, i64, i32, i32, i64, vp, i64, vp, vp, vp, vp]
        lib.oracle_build_leaves_ex.restype = i64
        lib.oracle_dtw64.argtypes = [vp, vp, i32, i32]
        lib.oracle_dtw64.restype = d
        lib.oracle_envelope.argtypes = [vp, i32, i32, vp, vp]
        lib.oracle_lb_keogh.argtypes = [vp, vp, vp, i32]
        lib.oracle_lb_keogh.restype = d
        lib.oracle_mindist_dtw_sq.argtypes = [vp, vp, i32, i32, vp, vp, i32, vp, d]
        lib.oracle_mindist_dtw_sq.restype = d
        lib.oracle_knn_brute_dtw.argtypes = [vp, i64, i32, vp, i32, i32, i32, ctypes.c_int, vp, vp]
        lib.oracle_knn_brute_dtw.restype = ctypes.c_int
        lib.oracle_knn_isax_dtw.argtypes = [vp, i64, i32, vp, i32, i32, vp, i64, vp, vp, i32, i32, i32, vp, vp, vp]
        lib.oracle_knn_isax_dtw.restype = ctypes.c_int
        lib.oracle_leaf_bounds.argtypes = [vp, i32, i32, i32, vp, i64, vp]
        lib.oracle_knn_approx.argtypes = [vp, i64, i32, i32, i32, vp, i64, vp, vp, i32, i32, i64, vp, vp, vp]
        lib.oracle_knn_approx.restype = ctypes.c_int
        lib.oracle_bf16_round_array.argtypes = [vp, i64, vp]
        lib.oracle_bf16_filter_values.argtypes = [vp, vp, i64, i32, vp]
        lib.oracle_bf16_error_bound.argtypes = [d, d, i32, vp]
        lib.oracle_bf16_error_bound.restype = d
        _lib = lib
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def breakpoints(card_bits: int) -> np.ndarray:
    """beta_j = fl32(Phi^-1(j / 2^b)), j = 1 .. 2^b - 1 (iSAX regions, Preliminaries)."""
    out = np.zeros(255, dtype=np.float32)
    cnt = _load().oracle_breakpoints(card_bits, out.ctypes.data)
    if cnt < 0:
        raise ValueError("card_bits must be in [1, 8]")
    return out[:cnt].copy()


def znorm(x) -> np.ndarray:
    """Per-series z-normalisation, fp64 statistics (Preliminaries)."""
    x = _f32(x)
    n, length = x.shape
    z = np.empty_like(x)
    _load().oracle_znorm(x.ctypes.data, n, length, z.ctypes.data)
    return z


def windows(long_series, length: int, step: int = 1, znorm_windows: bool = True) -> np.ndarray:
    """Subsequences of a streaming series by a sliding window (Preliminaries:
    the windows of the query length are what gets indexed): row r is
    long_series[r*step : r*step + length], for every r whose window fits,
    then z-normalised per window as any collection is."""
    x = _f32(long_series).ravel()
    if length < 1 or step < 1 or x.size < length:
        raise ValueError("need 1 <= length <= len(long_series) and step >= 1")
    count = (x.size - length) // step + 1
    rows = np.stack([x[r * step:r * step + length] for r in range(count)])
    return znorm(rows) if znorm_windows else rows


def paa(z, segments: int) -> np.ndarray:
    """Segment means, fp32, fold-halving order (PAA, Preliminaries)."""
    z = _f32(z)
    n, length = z.shape
    if length % segments:
        raise ValueError("length must be a multiple of segments")
    out = np.empty((n, segments), dtype=np.float32)
    _load().oracle_paa(z.ctypes.data, n, length, segments, out.ctypes.data)
    return out


def symbols(paa_values, card_bits: int) -> np.ndarray:
    """iSAX word: number of breakpoints <= each PAA value (Preliminaries)."""
    p = _f32(paa_values)
    n, w = p.shape
    bp = breakpoints(card_bits)
    full = np.zeros(255, dtype=np.float32)
    full[:bp.size] = bp
    out = np.empty((n, w), dtype=np.uint8)
    _load().oracle_symbols(p.ctypes.data, n, w, card_bits, full.ctypes.data, out.ctypes.data)
    return out


def words(z, segments: int, card_bits: int) -> np.ndarray:
    return symbols(paa(z, segments), card_bits)


def root_keys(words_, card_bits: int) -> np.ndarray:
    wd = np.ascontiguousarray(words_, dtype=np.uint8)
    n, w = wd.shape
    out = np.empty(n, dtype=np.uint32)
    _load().oracle_root_keys(wd.ctypes.data, n, w, card_bits, out.ctypes.data)
    return out


SPLIT_DTYPE = np.dtype([("card", np.uint8, (16,)), ("prefix", np.uint8, (16,)), ("seg", np.int32)])


def build_leaves(words_, card_bits: int, leaf_cap: int, forced=None, return_inner=False):
    """Leaf partition by the order-free top-down rule (TreeConstruction/SplitNode).

    forced: internal nodes (SPLIT_DTYPE) that must split on their segment --
    appending series to an index is the partition of all its series with the
    previous partition's internal nodes forced (see append_leaves).
    Returns (leaves structured array in depth-first order, pos uint32[n])
    and, with return_inner, the internal nodes with their segments."""
    wd = np.ascontiguousarray(words_, dtype=np.uint8)
    n, w = wd.shape
    leaves = np.zeros(n, dtype=LEAF_DTYPE)
    pos = np.zeros(n, dtype=np.uint32)
    f = np.ascontiguousarray(forced if forced is not None else np.zeros(0, SPLIT_DTYPE), dtype=SPLIT_DTYPE)
    inner = np.zeros((w * (card_bits - 1) + 2) * (n // (leaf_cap + 1) + 1), dtype=SPLIT_DTYPE)
    n_inner = ctypes.c_int64(0)
    cnt = _load().oracle_build_leaves_ex(wd.ctypes.data, n, w, card_bits, leaf_cap, f.ctypes.data, f.size,
                                         leaves.ctypes.data, pos.ctypes.data, inner.ctypes.data,
                                         ctypes.byref(n_inner))
    if cnt < 0:
        raise ValueError("bad arguments to build_leaves")
    out = (leaves[:cnt].copy(), pos)
    return out + (inner[:n_inner.value].copy(),) if return_inner else out


def append_leaves(words_all, card_bits: int, leaf_cap: int, inner_before):
    """The index after appending series (Algorithm TreeConstruction's insert
    and SplitNode): words_all holds the words of the old series followed by
    the new ones; every node that was internal before splits on the same
    segment, everything else follows the top-down rule.  Returns (leaves,
    pos, inner) of the new index."""
    return build_leaves(words_all, card_bits, leaf_cap, forced=inner_before, return_inner=True)


def d64(q, x) -> float:
    """Canonical squared ED: sequential fp64 sum, no fused multiply-add."""
    q, x = _f32(q), _f32(x)
    return _load().oracle_d64(q.ctypes.data, x.ctypes.data, q.size)


def mindist_sq(qpaa, card, prefix, card_bits: int, m: int, slack: float = 0.0) -> float:
    """iSAX MINDIST^2 of a (fp64) query PAA against a node region."""
    qp = np.ascontiguousarray(qpaa, dtype=np.float64)
    w = qp.size
    c = np.zeros(16, dtype=np.uint8); c[:w] = card
    p = np.zeros(16, dtype=np.uint8); p[:w] = prefix
    bp = np.zeros(255, dtype=np.float32)
    b = breakpoints(card_bits); bp[:b.size] = b
    return _load().oracle_mindist_sq(qp.ctypes.data, w, m, c.ctypes.data, p.ctypes.data, card_bits,
                                     bp.ctypes.data, float(slack))


def knn_brute(data, queries, k: int, nthreads: int = 1, row_offset: int = 0):
    """Exact k-NN by full scan: k smallest (D64, index), ascending.

    Returns (idx int64[nq, k], d64 float64[nq, k], dist float32[nq, k] = fl32(sqrt(D64)))."""
    data, queries = _f32(data), _f32(queries)
    n, length = data.shape
    nq = queries.shape[0]
    idx = np.zeros((nq, k), dtype=np.int64)
    dd = np.zeros((nq, k), dtype=np.float64)
    rc = _load().oracle_knn_brute(data.ctypes.data, n, length, queries.ctypes.data, nq, k, int(nthreads),
                                  int(row_offset), idx.ctypes.data, dd.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments to knn_brute")
    return idx, dd, np.sqrt(dd).astype(np.float32)


def knn_isax(data, words_, card_bits, leaves, pos, queries, k: int, return_stats=False):
    """Plain iSAX exact search over the oracle's own index (must equal knn_brute)."""
    data, queries = _f32(data), _f32(queries)
    wd = np.ascontiguousarray(words_, dtype=np.uint8)
    n, length = data.shape
    w = wd.shape[1]
    nq = queries.shape[0]
    leaves = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
    pos = np.ascontiguousarray(pos, dtype=np.uint32)
    idx = np.zeros((nq, k), dtype=np.int64)
    dd = np.zeros((nq, k), dtype=np.float64)
    stats = np.zeros((nq, 4), dtype=np.int64)
    rc = _load().oracle_knn_isax(data.ctypes.data, n, length, wd.ctypes.data, w, card_bits, leaves.ctypes.data,
                                 leaves.size, pos.ctypes.data, queries.ctypes.data, nq, k, idx.ctypes.data,
                                 dd.ctypes.data, stats.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments to knn_isax")
    out = (idx, dd, np.sqrt(dd).astype(np.float32))
    return out + (stats,) if return_stats else out


def dtw64(q, x, band: int) -> float:
    """Squared DTW under a Sakoe-Chiba band of half-width `band`, fp64, by the
    textbook recurrence (the paper's DTW experiment; Berndt & Clifford)."""
    q, x = _f32(q).ravel(), _f32(x).ravel()
    assert q.size == x.size
    return _load().oracle_dtw64(q.ctypes.data, x.ctypes.data, q.size, int(band))


def envelope(q, band: int):
    """LB_Keogh envelope of q over the band: (up, lo), fp32."""
    q = _f32(q).ravel()
    up, lo = np.empty_like(q), np.empty_like(q)
    _load().oracle_envelope(q.ctypes.data, q.size, int(band), up.ctypes.data, lo.ctypes.data)
    return up, lo


def lb_keogh(q, x, band: int) -> float:
    """LB_Keogh^2 of x against the envelope of q, fp64."""
    up, lo = envelope(q, band)
    x = _f32(x).ravel()
    return _load().oracle_lb_keogh(up.ctypes.data, lo.ctypes.data, x.ctypes.data, x.size)


def mindist_dtw_sq(q, band: int, card, prefix, card_bits: int, segments: int, slack: float = 0.0) -> float:
    """The index bound under DTW: per segment the envelope's max / min against
    the node's region (LB_PAA of the envelope), fp64."""
    up, lo = envelope(q, band)
    bp = np.zeros(255, dtype=np.float32)
    b = breakpoints(card_bits)
    bp[:b.size] = b
    c = np.zeros(16, np.uint8)
    p = np.zeros(16, np.uint8)
    c[:segments] = card[:segments]
    p[:segments] = prefix[:segments]
    return _load().oracle_mindist_dtw_sq(up.ctypes.data, lo.ctypes.data, up.size, segments, c.ctypes.data,
                                         p.ctypes.data, card_bits, bp.ctypes.data, float(slack))


def knn_brute_dtw(data, queries, k: int, band: int, nthreads: int = 1):
    """Exact k-NN under DTW by full scan: k smallest (DTW64, index).
    Returns (idx, dtw64, fl32(sqrt(dtw64)))."""
    data, queries = _f32(data), _f32(queries)
    n, length = data.shape
    nq = queries.shape[0]
    idx = np.zeros((nq, k), dtype=np.int64)
    dd = np.zeros((nq, k), dtype=np.float64)
    rc = _load().oracle_knn_brute_dtw(data.ctypes.data, n, length, queries.ctypes.data, nq, k, int(band),
                                      int(nthreads), idx.ctypes.data, dd.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments to knn_brute_dtw")
    return idx, dd, np.sqrt(dd).astype(np.float32)


def knn_isax_dtw(data, words_, card_bits, leaves, pos, queries, k: int, band: int, return_stats=False):
    """DTW k-NN through the oracle's index with the envelope bounds and
    LB_Keogh (must equal knn_brute_dtw)."""
    data, queries = _f32(data), _f32(queries)
    wd = np.ascontiguousarray(words_, dtype=np.uint8)
    n, length = data.shape
    w = wd.shape[1]
    nq = queries.shape[0]
    leaves = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
    pos = np.ascontiguousarray(pos, dtype=np.uint32)
    idx = np.zeros((nq, k), dtype=np.int64)
    dd = np.zeros((nq, k), dtype=np.float64)
    stats = np.zeros((nq, 4), dtype=np.int64)
    rc = _load().oracle_knn_isax_dtw(data.ctypes.data, n, length, wd.ctypes.data, w, card_bits, leaves.ctypes.data,
                                     leaves.size, pos.ctypes.data, queries.ctypes.data, nq, k, int(band),
                                     idx.ctypes.data, dd.ctypes.data, stats.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments to knn_isax_dtw")
    out = (idx, dd, np.sqrt(dd).astype(np.float32))
    return out + (stats,) if return_stats else out


def leaf_bounds(query, segments: int, card_bits: int, leaves) -> np.ndarray:
    """MINDIST^2 (fp64, no widening) of one query's PAA to every leaf's regions."""
    q = _f32(query).ravel()
    leaves = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
    out = np.zeros(leaves.size, dtype=np.float64)
    _load().oracle_leaf_bounds(q.ctypes.data, q.size, segments, card_bits, leaves.ctypes.data, leaves.size,
                               out.ctypes.data)
    return out


def knn_approx(data, segments: int, card_bits: int, leaves, pos, queries, k: int, leaf=None):
    """The paper's approximate search (Section 4, approxSearch): the k best
    members of the leaf with the smallest bound (or of `leaf`), extended in
    depth-first order to at least k members, at most 4096.
    Returns (leaf int64[nq], idx int64[nq, k], d64 float64[nq, k], dist float32[nq, k])."""
    data, queries = _f32(data), _f32(queries)
    n, length = data.shape
    nq = queries.shape[0]
    leaves = np.ascontiguousarray(leaves, dtype=LEAF_DTYPE)
    pos = np.ascontiguousarray(pos, dtype=np.uint32)
    lf = np.zeros(nq, dtype=np.int64)
    idx = np.zeros((nq, k), dtype=np.int64)
    dd = np.zeros((nq, k), dtype=np.float64)
    rc = _load().oracle_knn_approx(data.ctypes.data, n, length, segments, card_bits, leaves.ctypes.data,
                                   leaves.size, pos.ctypes.data, queries.ctypes.data, nq, k,
                                   -1 if leaf is None else int(leaf), lf.ctypes.data, idx.ctypes.data,
                                   dd.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments to knn_approx")
    return lf, idx, dd, np.sqrt(dd).astype(np.float32)


def bf16_round(v) -> np.ndarray:
    """Round fp32 values to BF16 (nearest, ties to even), returned as fp32."""
    a = _f32(v)
    out = np.empty_like(a)
    _load().oracle_bf16_round_array(a.ctypes.data, a.size, out.ctypes.data)
    return out


def bf16_filter_values(q, x) -> np.ndarray:
    """Filtered squared distance of each row pair (q[i], x[i]) as the BF16
    filter of the batched search defines it: fl32(fl32(|q|^2 + |x|^2) - 2 s),
    s the fp32 sum in index order of the exact BF16 products."""
    q2, x2 = _f32(q), _f32(x)
    assert q2.shape == x2.shape and q2.ndim == 2
    out = np.empty(q2.shape[0], dtype=np.float32)
    _load().oracle_bf16_filter_values(q2.ctypes.data, x2.ctypes.data, q2.shape[0], q2.shape[1], out.ctypes.data)
    return out


def bf16_error_bound(norm2_q: float, norm2_x: float, length: int, terms: bool = False):
    """Bound E on |f - D| for the BF16 filter (any order and rounding of its
    fp32 accumulation).  With terms=True also returns the five parts:
    operands, accumulation, norms, first add, final subtraction."""
    t = np.zeros(5, dtype=np.float64)
    e = _load().oracle_bf16_error_bound(float(norm2_q), float(norm2_x), int(length), t.ctypes.data)
    return (e, t) if terms else e
