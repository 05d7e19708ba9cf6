"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Bars: iSAX words, leaf records, member order and neighbour indices bit-exact;
z-normalised values bit-exact (same fp64 statistics in the same order);
distances within 1e-5 relative of the oracle's fp64 distance.
All calls go through the C ABI (ctypes binding)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def messi():
    from paper_2009_00786_amd import messi as m
    m.load()
    return m


def _say(*a):
    print(*a, flush=True)


def gpu_walks(torch, dg, n, length, seed, stream, row0=0):
    t = torch.empty((n, length), dtype=torch.float32, device="cuda")
    dg.gpu_random_walks(t, seed=seed, stream=stream, row0=row0)
    return t


# ---------------------------------------------------------------------------
# generator and z-normalisation
# ---------------------------------------------------------------------------

def test_gpu_generator_matches_host(torch_cuda, datagen_mod):
    torch = torch_cuda
    _say("generator: walks 20000x256, mixture 3000x128")
    g = gpu_walks(torch, datagen_mod, 20000, 256, 2009, 0).cpu().numpy()
    h = datagen_mod.random_walks(20000, 256, seed=2009, stream=0)
    np.testing.assert_array_equal(g, h)
    cen = datagen_mod.mixture_centres(1000, 128)
    gm = torch.empty((3000, 128), dtype=torch.float32, device="cuda")
    datagen_mod.gpu_mixture(gm, torch.from_numpy(cen).cuda(), row0=12345)
    hm = datagen_mod.mixture(3000, 128, cen, row0=12345)
    np.testing.assert_array_equal(gm.cpu().numpy(), hm)


# 1M x 256 makes the fp64 quotient land near an fp32 rounding midpoint a few
# times, so both ways of forming the fp32 quotient are exercised
@pytest.mark.parametrize("n,length", [(1_000_000, 256), (100_000, 256), (4097, 128), (3001, 96), (1000, 100),
                                      (777, 1000), (300, 512), (200, 33), (500, 16), (33, 3), (1, 64)])
def test_znorm_bitwise(torch_cuda, messi, datagen_mod, oracle_mod, n, length):
    torch = torch_cuda
    _say("znorm n=%d len=%d" % (n, length))
    x = datagen_mod.random_walks(n, length, seed=77, stream=0)
    x[n // 2] = 3.5  # a constant series -> zeros
    t = torch.from_numpy(x).cuda()
    messi.znorm_(t)
    np.testing.assert_array_equal(t.cpu().numpy(), oracle_mod.znorm(x))


# ---------------------------------------------------------------------------
# index build: words, leaves, member order
# ---------------------------------------------------------------------------

BUILD_CASES = [
    # n, len, segments, bits, cap
    (100_000, 256, 16, 8, 2000),   # the tiny workload of the paper's setup
    (12289, 128, 16, 8, 100),      # ragged last tile, two series per wave
    (700, 64, 16, 8, 20),          # fewer rows than one radix sub-tile (1024)
    (4097, 64, 8, 8, 10),
    (3000, 96, 16, 8, 50),         # segment length 6: padded fold-halving path
    (2000, 100, 4, 4, 20),         # length not a power of two, segment length 25
    (5000, 256, 4, 1, 50),         # one bit per symbol: no splits possible
    (3000, 1024, 16, 8, 300),      # longest supported rows
    (50, 32, 2, 8, 1000),          # capacity above n: leaves = root children
    (7, 16, 16, 3, 1),
    (1, 16, 4, 8, 10),
]


def test_znorm_adversarial_orders(torch_cuda, messi, oracle_mod):
    """Rows whose fp64 statistics depend on the summation order (values
    spread beyond fp64's 53 bits): the GPU's fold-halving sums must give the
    oracle's result bit for bit."""
    torch = torch_cuda
    _say("z-norm: order-sensitive rows")
    for L in (4, 6, 64, 256, 1000):
        x = np.zeros((5, L), dtype=np.float32)
        x[0, 0], x[0, 1 % L], x[0, L // 2], x[0, (L // 2 + 1) % L] = 2.0 ** 60, 1.0, -(2.0 ** 60), 1.0
        x[1, :] = 1.0
        x[1, 0], x[1, L - 1] = 2.0 ** 70, -(2.0 ** 70)
        x[2, ::2] = 2.0 ** 40
        x[2, 1::2] = 3.0
        x[3] = np.arange(L, dtype=np.float32) * np.float32(2.0 ** 30) + 1.0
        x[4, 0] = 1.0
        t = torch.from_numpy(x.copy()).cuda()
        messi.znorm_(t)
        np.testing.assert_array_equal(t.cpu().numpy(), oracle_mod.znorm(x))


def _oracle_index(oracle_mod, z, w, b, cap):
    words = oracle_mod.words(z, w, b)
    leaves, pos = oracle_mod.build_leaves(words, b, cap)
    return words, leaves, pos


@pytest.mark.parametrize("n,length,w,b,cap", BUILD_CASES)
def test_build_bitwise(torch_cuda, messi, datagen_mod, oracle_mod, n, length, w, b, cap):
    torch = torch_cuda
    _say("build n=%d len=%d w=%d b=%d cap=%d" % (n, length, w, b, cap))
    x = datagen_mod.random_walks(n, length, seed=2009, stream=0)
    z = oracle_mod.znorm(x)
    t = torch.from_numpy(x).cuda()
    ix = messi.Index(t, segments=w, card_bits=b, leaf_cap=cap, znorm=True)
    # the fused z-normalisation wrote the same values as the oracle
    np.testing.assert_array_equal(t.cpu().numpy(), z)
    ow, ol, op = _oracle_index(oracle_mod, z, w, b, cap)
    np.testing.assert_array_equal(ix.export_words(), ow)
    gl, gp = ix.export_leaves()
    assert len(gl) == len(ol)
    np.testing.assert_array_equal(gl["card"], ol["card"])
    np.testing.assert_array_equal(gl["prefix"], ol["prefix"])
    np.testing.assert_array_equal(gl["start"], ol["start"])
    np.testing.assert_array_equal(gl["count"], ol["count"])
    np.testing.assert_array_equal(gp, op)
    info = ix.info()
    assert info["n_leaves"] == len(ol) and info["max_leaf"] == int(ol["count"].max())
    ix.close()


def test_build_with_duplicates_and_overflow_leaves(torch_cuda, messi, oracle_mod):
    torch = torch_cuda
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3000, 64)).astype(np.float32)
    x[100:1200] = x[5]            # > cap identical series -> an overflow leaf
    x[2000:2010] = 1.0            # constant series
    z = oracle_mod.znorm(x)
    t = torch.from_numpy(z.copy()).cuda()
    ix = messi.Index(t, segments=8, card_bits=8, leaf_cap=100)
    ow, ol, op = _oracle_index(oracle_mod, z, 8, 8, 100)
    np.testing.assert_array_equal(ix.export_words(), ow)
    gl, gp = ix.export_leaves()
    np.testing.assert_array_equal(gl["start"], ol["start"])
    np.testing.assert_array_equal(gl["count"], ol["count"])
    np.testing.assert_array_equal(gl["card"], ol["card"])
    np.testing.assert_array_equal(gp, op)
    assert ol["count"].max() > 100


# ---------------------------------------------------------------------------
# exact k-NN
# ---------------------------------------------------------------------------

def _check_answers(gidx, gdist, oidx, od64):
    np.testing.assert_array_equal(gidx, oidx)
    ref = np.sqrt(od64)
    err = np.abs(gdist.astype(np.float64) - ref) / np.maximum(ref, 1e-30)
    assert np.all((err <= REL_TOL) | (ref == 0) & (gdist == 0)), float(err.max())


@pytest.fixture(scope="module")
def tiny_workload(torch_cuda, messi, datagen_mod, oracle_mod):
    """100,000 z-normalised random walks of length 256 (16 segments, 8 bits,
    leaf capacity 2000) and 10 fresh walks as queries."""
    torch = torch_cuda
    x = datagen_mod.random_walks(100_000, 256)
    z = oracle_mod.znorm(x)
    t = torch.from_numpy(x).cuda()
    ix = messi.Index(t, 16, 8, 2000, znorm=True)
    qr = datagen_mod.random_walks(10, 256, seed=datagen_mod.SEED_QUERY, stream=datagen_mod.STREAM_QUERY)
    qz = oracle_mod.znorm(qr)
    qt = torch.from_numpy(qr).cuda()
    messi.znorm_(qt)
    np.testing.assert_array_equal(qt.cpu().numpy(), qz)
    yield {"z": z, "ix": ix, "qz": qz, "qt": qt}
    ix.close()


def test_knn_single_queries_k1(tiny_workload, oracle_mod):
    w = tiny_workload
    _say("knn tiny workload, single queries, k=1")
    oidx, od, _ = oracle_mod.knn_brute(w["z"], w["qz"], 1, nthreads=8)
    for i in range(10):
        gi, gd = w["ix"].knn(w["qt"][i:i + 1], 1)
        _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx[i:i + 1], od[i:i + 1])


@pytest.mark.parametrize("k", [1, 2, 10, 100])
def test_knn_batched(tiny_workload, oracle_mod, datagen_mod, torch_cuda, k):
    torch = torch_cuda
    w = tiny_workload
    _say("knn tiny workload, batched, k=%d" % k)
    rows = datagen_mod.uniform_ints(6, 100_000, 9, 5)
    qn = datagen_mod.add_noise(w["z"][rows], [0.01, 0.1, 1.0, 0.01, 0.1, 1.0])
    q = np.concatenate([w["qz"], qn])
    oidx, od, _ = oracle_mod.knn_brute(w["z"], q, k, nthreads=8)
    gi, gd, st = w["ix"].knn(torch.from_numpy(q).cuda(), k, stats=True)
    _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx, od)
    assert st["series_distance"] < 100_000 * len(q)  # pruning happened
    _say("  stats", st)


def test_plain_messi_knn_entry_point(tiny_workload, oracle_mod):
    """messi_knn itself: synchronous, the index's default mode (FP32), one query
    and a batch."""
    w = tiny_workload
    _say("messi_knn: single queries k=1 and a batch k=5")
    oidx, od, _ = oracle_mod.knn_brute(w["z"], w["qz"], 5, nthreads=8)
    for i in range(3):
        gi, gd = w["ix"].knn_plain(w["qt"][i:i + 1].contiguous(), 1)
        _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx[i:i + 1, :1], od[i:i + 1, :1])
    gi, gd = w["ix"].knn_plain(w["qt"], 5)
    _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx, od)


@pytest.fixture(scope="module")
def tiny_bf16_index(tiny_workload, torch_cuda, messi):
    """A second index over the same rows with the BF16 shadow."""
    t = torch_cuda.from_numpy(tiny_workload["z"]).cuda()
    ix = messi.Index(t, 16, 8, 2000, bf16_shadow=True)
    yield ix
    ix.close()


@pytest.mark.parametrize("mode_name", ["FP32", "BF16"])
def test_knn_per_query_k(tiny_workload, tiny_bf16_index, oracle_mod, datagen_mod, torch_cuda, messi, mode_name):
    """messi_knn_ex with k_per_query: row q holds the k_per_query[q] nearest
    neighbours of query q, then (-1, +inf) up to k_max."""
    torch = torch_cuda
    w = tiny_workload
    rows = datagen_mod.uniform_ints(10, 100_000, 19, 5)
    qn = datagen_mod.add_noise(w["z"][rows], [0.01, 0.1, 1.0, 0.01, 0.1, 1.0, 0.01, 0.1, 1.0, 0.5])
    q = np.concatenate([w["qz"], qn])
    ks = np.array([1, 7, 100, 3, 1, 50, 10, 2, 64, 1, 100, 5, 1, 33, 9, 2, 17, 1, 80, 4], dtype=np.int32)
    kmax = 100
    mode = messi.MODE_BF16 if mode_name == "BF16" else messi.MODE_FP32
    _say("per-query k, %s, %d queries, k_max %d" % (mode_name, len(q), kmax))
    oidx, od, _ = oracle_mod.knn_brute(w["z"], q, kmax, nthreads=8)
    gi, gd = tiny_bf16_index.knn(torch.from_numpy(q).cuda(), kmax, mode=mode,
                                 k_per_query=torch.from_numpy(ks).cuda())
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    for i, kq in enumerate(ks):
        _check_answers(gi[i:i + 1, :kq], gd[i:i + 1, :kq], oidx[i:i + 1, :kq], od[i:i + 1, :kq])
        assert np.all(gi[i, kq:] == -1) and np.all(np.isposinf(gd[i, kq:]))
    # a k outside [1, k_max] is rejected before any search
    bad = torch.from_numpy(np.array([1, 0], dtype=np.int32)).cuda()
    with pytest.raises(messi.MessiError) as e:
        tiny_bf16_index.knn(torch.from_numpy(q[:2].copy()).cuda(), 4, k_per_query=bad)
    assert e.value.code == messi.MESSI_EINVAL
    bad = torch.from_numpy(np.array([5, 1], dtype=np.int32)).cuda()
    with pytest.raises(messi.MessiError) as e:
        tiny_bf16_index.knn(torch.from_numpy(q[:2].copy()).cuda(), 4, k_per_query=bad)
    assert e.value.code == messi.MESSI_EINVAL


@pytest.mark.parametrize("chunk", [256, 512])
def test_index_options_scan_chunk_and_mode(tiny_workload, oracle_mod, datagen_mod, torch_cuda, messi, chunk):
    """Index options: a smaller scan chunk gives the same exact answers, and
    messi_knn runs in the index's own mode (BF16 here)."""
    torch = torch_cuda
    w = tiny_workload
    t = torch.from_numpy(w["z"]).cuda()
    ix = messi.Index(t, 16, 8, 2000, bf16_shadow=True, scan_chunk=chunk, mode=messi.MODE_BF16)
    rows = datagen_mod.uniform_ints(4, 100_000, 23, 5)
    q = np.concatenate([w["qz"][:4], datagen_mod.add_noise(w["z"][rows], [0.01, 0.1, 1.0, 0.3])])
    for k in (1, 10):
        _say("scan chunk %d, k=%d: FP32 one at a time, messi_knn (BF16) batched" % (chunk, k))
        oidx, od, _ = oracle_mod.knn_brute(w["z"], q, k, nthreads=8)
        for i in range(len(q)):
            gi, gd = ix.knn(torch.from_numpy(q[i:i + 1].copy()).cuda(), k)
            _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx[i:i + 1], od[i:i + 1])
        gi, gd = ix.knn_plain(torch.from_numpy(q).cuda(), k)
        _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx, od)
    ix.close()


def test_workspace_budget(tiny_workload, torch_cuda, messi):
    """budget_bytes caps a stream's search workspace: a call that needs more
    fails with MESSI_ENOMEM; a large enough budget answers as usual."""
    w = tiny_workload
    t = torch_cuda.from_numpy(w["z"]).cuda()
    small = messi.Index(t, 16, 8, 2000, budget_bytes=1 << 20)
    with pytest.raises(messi.MessiError) as e:
        small.knn(w["qt"][:1].contiguous(), 1)
    assert e.value.code == messi.MESSI_ENOMEM
    small.close()
    big = messi.Index(t, 16, 8, 2000, budget_bytes=64 << 20)
    a = big.knn(w["qt"][:2].contiguous(), 3)
    b = w["ix"].knn(w["qt"][:2].contiguous(), 3)
    assert torch_cuda.equal(a[0], b[0]) and torch_cuda.equal(a[1], b[1])
    big.close()


def test_knn_matches_oracle_isax_counts(tiny_workload, oracle_mod):
    """The oracle's pruned search and the GPU give the same answers."""
    w = tiny_workload
    words = oracle_mod.words(w["z"], 16, 8)
    leaves, pos = oracle_mod.build_leaves(words, 8, 2000)
    oi, od, _ = oracle_mod.knn_isax(w["z"], words, 8, leaves, pos, w["qz"][:3], 5)
    gi, gd = w["ix"].knn(w["qt"][:3].contiguous(), 5)
    _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oi, od)


KNN_EDGE = [
    # n, len, w, b, cap, k
    (1, 16, 4, 8, 10, 1),
    (7, 16, 16, 3, 1, 7),          # k = n
    (64, 32, 8, 8, 4, 64),
    (4097, 64, 8, 8, 10, 3),
    (3000, 96, 16, 8, 50, 5),
    (2000, 100, 4, 4, 20, 4),      # scalar row path
    (5000, 256, 4, 1, 50, 2),
    (3000, 1024, 16, 8, 300, 1),
    (12289, 128, 16, 8, 2000, 17),
]


@pytest.mark.parametrize("n,length,w,b,cap,k", KNN_EDGE)
def test_knn_shapes(torch_cuda, messi, datagen_mod, oracle_mod, n, length, w, b, cap, k):
    torch = torch_cuda
    _say("knn n=%d len=%d w=%d b=%d cap=%d k=%d" % (n, length, w, b, cap, k))
    z = oracle_mod.znorm(datagen_mod.random_walks(n, length, seed=31, stream=0))
    q = oracle_mod.znorm(datagen_mod.random_walks(4, length, seed=32, stream=1))
    q = np.concatenate([q, z[[0, n - 1]]])
    t = torch.from_numpy(z).cuda()
    ix = messi.Index(t, w, b, cap)
    oidx, od, _ = oracle_mod.knn_brute(z, q, k, nthreads=8)
    gi, gd = ix.knn(torch.from_numpy(q).cuda(), k)
    _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx, od)
    for i in range(len(q)):  # one query at a time, too
        gi1, gd1 = ix.knn(torch.from_numpy(q[i:i + 1]).cuda(), k)
        _check_answers(gi1.cpu().numpy(), gd1.cpu().numpy(), oidx[i:i + 1], od[i:i + 1])
    ix.close()


def test_knn_ties_and_degenerate(torch_cuda, messi, oracle_mod):
    torch = torch_cuda
    _say("knn ties and degenerate series")
    rng = np.random.default_rng(7)
    z = oracle_mod.znorm(rng.standard_normal((3000, 64)).astype(np.float32))
    z[100:400] = z[7]             # 301 identical rows (overflow leaf at cap 50)
    z[500:520] = 0.0              # constant series
    q = np.concatenate([z[[7, 500, 2999]], rng.standard_normal((2, 64)).astype(np.float32)])
    t = torch.from_numpy(z).cuda()
    ix = messi.Index(t, 8, 8, 50)
    for k in (1, 5, 40, 350):
        oidx, od, _ = oracle_mod.knn_brute(z, q, k, nthreads=8)
        gi, gd = ix.knn(torch.from_numpy(q).cuda(), k)
        _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx, od)
    gi, gd = ix.knn(torch.from_numpy(z[150:151].copy()).cuda(), 3)
    assert list(gi.cpu().numpy()[0]) == [7, 100, 101]


def test_knn_candidate_overflow_recovers(torch_cuda, messi, datagen_mod, oracle_mod):
    """A candidate buffer far smaller than what a loose first bound lets
    through: the scan reruns from the k-th buffered distance (and the call
    retries with a larger buffer if even that overflows); answers stay exact."""
    torch = torch_cuda
    z = oracle_mod.znorm(datagen_mod.random_walks(30_000, 64, seed=77, stream=0))
    q = datagen_mod.add_noise(z[[5, 17_000, 29_999]], [1.0, 1.0, 0.5])
    ix = messi.Index(torch.from_numpy(z).cuda(), 16, 8, 200, cand_cap=64)
    reruns = 0
    for k in (1, 8, 30):
        _say("overflow recovery k=%d" % k)
        oidx, od, _ = oracle_mod.knn_brute(z, q, k, nthreads=8)
        gi, gd, st = ix.knn(torch.from_numpy(q).cuda(), k, stats=True)
        _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx, od)
        reruns += st["reruns"]
        gi, gd, st = ix.knn(torch.from_numpy(q[:1].copy()).cuda(), k, stats=True)
        _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx[:1], od[:1])
        reruns += st["reruns"]
        # one query without statistics: its error flag comes back through
        # host memory instead of a copy, retries included
        gi, gd = ix.knn(torch.from_numpy(q[:1].copy()).cuda(), k)
        _check_answers(gi.cpu().numpy(), gd.cpu().numpy(), oidx[:1], od[:1])
    assert reruns > 0
    ix.close()


def test_knn_nq_zero_and_errors(torch_cuda, messi):
    torch = torch_cuda
    z = torch.randn((100, 32), device="cuda")
    messi.znorm_(z)
    ix = messi.Index(z, 4, 8, 10)
    empty = torch.empty((0, 32), device="cuda")
    gi, gd = ix.knn(empty, 1)
    assert gi.shape == (0, 1)
    with pytest.raises(messi.MessiError) as e:
        ix.knn(z[:1].contiguous(), 101)
    assert e.value.code == messi.MESSI_EINVAL
    bad = z[:1].clone()
    bad[0, 3] = float("nan")
    with pytest.raises(messi.MessiError) as e:
        ix.knn(bad, 1)
    assert e.value.code == messi.MESSI_EINVAL
    import ctypes
    host = np.zeros((1, 32), dtype=np.float32)
    out_i = torch.empty((1, 1), dtype=torch.int64, device="cuda")
    out_d = torch.empty((1, 1), dtype=torch.float32, device="cuda")
    rc = messi.load().messi_knn(ix.handle, ctypes.c_void_p(host.ctypes.data), 1, 1,
                                ctypes.c_void_p(out_i.data_ptr()), ctypes.c_void_p(out_d.data_ptr()))
    assert rc == messi.MESSI_EINVAL
    x = torch.randn((50, 32), device="cuda")
    x[3, 3] = float("inf")
    with pytest.raises(messi.MessiError) as e:
        messi.Index(x, 4, 8, 10)
    assert e.value.code == messi.MESSI_EINVAL
    with pytest.raises(messi.MessiError):
        messi.Index(x, 5, 8, 10)   # 32 % 5 != 0
    ix.close()


# ---------------------------------------------------------------------------
# approximate mode (the paper's approxSearch)
# ---------------------------------------------------------------------------

def _lb_window(z, q, w, lb):
    """How far the GPU's leaf bound can lie from the oracle's, per leaf.

    The GPU bounds a leaf in fp32 from the query's fp32 PAA p' against
    regions widened by delta (the slack that keeps its bound below the exact
    distance); the oracle uses the fp64 PAA p and the plain regions.  The gap
    to an interval is 1-Lipschitz in the point and shrinks by at most delta
    when the interval widens by delta, so per segment the GPU's gap g_i and
    the oracle's d_i differ by at most |p' - p| + delta <= 2 delta (delta
    covers the fp32 PAA error of the query), and with LB = m sum d_i^2:
        |LB_gpu - LB| <= m sum 2 delta (2 d_i + 2 delta) + fp32 rounding
                      <= 4 m delta (sum d_i + w delta) + (w + 3) 2^-24 LB,
    where sum d_i <= sqrt(w LB / m).  delta is the GPU's: 1.01 (2 (lg m + 1) u
    A_data + 2 (m + 1) u A_q), u = 2^-24."""
    L = q.size
    m = L // w
    lg = int(math.ceil(math.log2(m))) if m > 1 else 0
    u = 2.0 ** -24
    delta = 1.01 * (2 * (lg + 1) * u * float(np.abs(z).max()) + 2 * (m + 1) * u * float(np.abs(q).max()))
    lb = np.asarray(lb, dtype=np.float64)
    return 4 * m * delta * (np.sqrt(w * lb / m) + w * delta) + (w + 3) * u * lb * 1.01


def _approx_matches(oracle_mod, z, leaves, pos, w, b, q, k, gi, gd):
    """The GPU's approximate answer is the oracle's for the leaf of smallest
    bound -- or, where two leaves' bounds are closer than the GPU's fp32
    bound can resolve (_lb_window), for the other leaf."""
    lf, oi, _, od = oracle_mod.knn_approx(z, w, b, leaves, pos, q[None, :], k)
    if np.array_equal(gi, oi[0]) and np.array_equal(gd, od[0]):
        return True
    lb = oracle_mod.leaf_bounds(q, w, b, leaves)
    win = _lb_window(z, q, w, lb)
    best = int(np.argmin(lb))
    near = np.nonzero(lb <= lb[best] + win + win[best])[0]
    for l in near:
        _, oi, _, od = oracle_mod.knn_approx(z, w, b, leaves, pos, q[None, :], k, leaf=int(l))
        if np.array_equal(gi, oi[0]) and np.array_equal(gd, od[0]):
            return True
    return False


@pytest.mark.parametrize("k", [1, 10, 100])
def test_approx_mode_matches_oracle(tiny_workload, oracle_mod, messi, torch_cuda, k):
    w = tiny_workload
    _say("approximate mode, tiny workload, k=%d (single and batched)" % k)
    leaves, pos = w["ix"].export_leaves()
    bi, bd = w["ix"].knn(w["qt"], k, mode=messi.MODE_APPROX)
    bi, bd = bi.cpu().numpy(), bd.cpu().numpy()
    ei, ed, _ = oracle_mod.knn_brute(w["z"], w["qz"], k, nthreads=8)
    for i in range(len(w["qz"])):
        si, sd = w["ix"].knn(w["qt"][i:i + 1], k, mode=messi.MODE_APPROX)
        np.testing.assert_array_equal(si.cpu().numpy()[0], bi[i])
        np.testing.assert_array_equal(sd.cpu().numpy()[0], bd[i])
        assert _approx_matches(oracle_mod, w["z"], leaves, pos, 16, 8, w["qz"][i], k, bi[i], bd[i]), i
        assert np.all(bd[i] >= np.sqrt(ed[i]).astype(np.float32))


def test_approx_mode_shapes(torch_cuda, messi, datagen_mod, oracle_mod):
    for (n, length, w, b, cap, k) in [(3000, 96, 8, 8, 50, 5), (500, 32, 16, 3, 7, 40), (64, 16, 4, 8, 1000, 64)]:
        _say("approximate mode n=%d L=%d w=%d b=%d cap=%d k=%d" % (n, length, w, b, cap, k))
        x = datagen_mod.random_walks(n, length, seed=n + 5)
        z = oracle_mod.znorm(x)
        q = oracle_mod.znorm(datagen_mod.random_walks(4, length, seed=n + 6, stream=1))
        ix = messi.Index(torch_cuda.from_numpy(z).cuda(), w, b, cap)
        leaves, pos = ix.export_leaves()
        gi, gd = ix.knn(torch_cuda.from_numpy(q).cuda(), k, mode=messi.MODE_APPROX)
        gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
        for i in range(len(q)):
            assert _approx_matches(oracle_mod, z, leaves, pos, w, b, q[i], k, gi[i], gd[i]), (n, i)
        ix.close()
