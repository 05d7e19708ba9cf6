"""Parity at the full workload size: 100M random walks of length 256 (102.4 GB
fp32 in HBM), 16 segments, 8-bit symbols, leaf capacity 2000 -- the index the
benchmark builds, in the same launch configuration.

The complete comparison (test_fullsize_against_oracle): the raw collection is
regenerated chunk by chunk, z-normalised and summarised by the oracle on the
host (every word compared), the oracle partitions all 100M words (every leaf
record and the whole position array compared), and the oracle's brute force
over all 100M rows answers the 100 queries the benchmark times (one at a time
on the GPU, exact 1-NN): indices bit-exact, distances those of fp64.

Beyond that, sampled outputs and properties that hold at any size:
  * iSAX words of 4096 random rows, each regenerated on the host and
    z-normalised and summarised by the oracle: bit-exact;
  * the leaves partition the collection (every series once, ranges
    contiguous in leaf order), and 500 random leaves hold exactly the members
    their (cardinality, prefix) describe, in ascending series order, within
    the capacity unless at full cardinality;
  * a dataset row used as the query is its own nearest neighbour at distance
    0 (no other row equals it); for fresh walks the returned distances are
    the oracle's canonical fp64 distances of the returned rows, no row of a
    1M-row block beats the returned k-th distance, and the BF16 batch returns
    the same answers as the FP32 single-query path, bit for bit."""
import concurrent.futures
import os
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 100_000_000
L = 256
CHUNK = 10_000_000


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


def _host_rows(dg, oracle, rows):
    """Raw rows regenerated on the host, z-normalised by the oracle."""
    raw = np.concatenate([dg.random_walks(1, L, row0=int(r)) for r in rows], axis=0)
    return oracle.znorm(raw)


@pytest.fixture(scope="module")
def full(torch_cuda, messi, datagen_mod):
    torch = torch_cuda
    _say("full size: generating %d x %d random walks on the GPU" % (N, L))
    data = torch.empty((N, L), dtype=torch.float32, device="cuda")
    for r0 in range(0, N, CHUNK):
        datagen_mod.gpu_random_walks(data[r0:r0 + CHUNK], row0=r0)
    messi.znorm_(data)
    torch.cuda.synchronize()
    _say("full size: building the index (with the BF16 shadow)")
    ix = messi.Index(data, 16, 8, 2000, bf16_shadow=True)
    yield {"data": data, "ix": ix}
    ix.close()
    del data
    torch.cuda.empty_cache()


def test_fullsize_words_sampled(full, datagen_mod, oracle_mod):
    rows = np.unique(datagen_mod.uniform_ints(4096, N, 71, 5))
    _say("full size: words of %d sampled rows" % len(rows))
    words = full["ix"].export_words()
    want = oracle_mod.words(_host_rows(datagen_mod, oracle_mod, rows), 16, 8)
    np.testing.assert_array_equal(words[rows], want)


def test_fullsize_leaves(full, datagen_mod):
    _say("full size: leaf partition and 500 sampled leaves")
    leaves, pos = full["ix"].export_leaves()
    counts = leaves["count"].astype(np.int64)
    starts = leaves["start"].astype(np.int64)
    assert counts.sum() == N
    assert starts[0] == 0 and np.all(starts[1:] == starts[:-1] + counts[:-1])
    seen = np.zeros(N, dtype=bool)
    seen[pos] = True
    assert seen.all()  # with the counts summing to N: every series exactly once
    words = full["ix"].export_words()
    pick = np.unique(datagen_mod.uniform_ints(500, len(leaves), 72, 5))
    for li in pick:
        lf = leaves[li]
        members = pos[lf["start"]:lf["start"] + lf["count"]].astype(np.int64)
        assert np.all(np.diff(members) > 0)
        w = words[members]
        card = lf["card"].astype(np.int32)
        for s in range(16):
            assert np.all((w[:, s] >> (8 - card[s])) == lf["prefix"][s])
        if lf["count"] > 2000:
            assert np.all(card == 8) and np.all(w == w[0])


@pytest.mark.parametrize("k", [1, 10])
def test_fullsize_knn(full, datagen_mod, oracle_mod, messi, torch_cuda, k):
    torch = torch_cuda
    ix = full["ix"]
    own = np.unique(datagen_mod.uniform_ints(6, N, 73, 5))
    q_rows = _host_rows(datagen_mod, oracle_mod, own)
    fresh = oracle_mod.znorm(datagen_mod.random_walks(6, L, seed=datagen_mod.SEED_QUERY,
                                                      stream=datagen_mod.STREAM_QUERY, row0=500))
    queries = np.concatenate([q_rows, fresh], axis=0).astype(np.float32)
    nq = len(queries)
    _say("full size: %d queries, k=%d, FP32 one at a time and one BF16 batch" % (nq, k))
    idx = np.zeros((nq, k), dtype=np.int64)
    dist = np.zeros((nq, k), dtype=np.float32)
    for i in range(nq):
        ai, ad = ix.knn(torch.from_numpy(queries[i:i + 1].copy()).cuda(), k)
        idx[i], dist[i] = ai.cpu().numpy()[0], ad.cpu().numpy()[0]
    bi, bd = ix.knn(torch.from_numpy(queries).cuda(), k, mode=messi.MODE_BF16)
    np.testing.assert_array_equal(bi.cpu().numpy(), idx)
    np.testing.assert_array_equal(bd.cpu().numpy(), dist)
    # a dataset row is its own nearest neighbour
    for j, r in enumerate(own):
        assert idx[j, 0] == r and dist[j, 0] == 0.0
    # returned distances are the canonical fp64 ones of the returned rows
    ret = np.unique(idx.ravel())
    ret_rows = dict(zip(ret.tolist(), _host_rows(datagen_mod, oracle_mod, ret)))
    for i in range(nq):
        for j in range(k):
            d64 = oracle_mod.d64(queries[i], ret_rows[int(idx[i, j])])
            assert dist[i, j] == np.float32(np.sqrt(d64)), (i, j)
        assert np.all(np.diff(dist[i]) >= 0)
    # no row of a 1M-row block beats the k-th returned distance
    r0 = 37_000_000
    block = oracle_mod.znorm(datagen_mod.random_walks(1_000_000, L, row0=r0))
    bi_, _, bdist = oracle_mod.knn_brute(block, queries, k, nthreads=16, row_offset=r0)
    for i in range(nq):
        assert bdist[i, k - 1] >= dist[i, k - 1]
        inside = (idx[i] >= r0) & (idx[i] < r0 + 1_000_000)
        # a global answer that lies in the block is among the block's own k best
        for j in np.nonzero(inside)[0]:
            assert idx[i, j] in bi_[i]


def _host_threads():
    """The host share a one-GPU job gets (16 threads), fewer on a smaller host."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def test_fullsize_against_oracle(full, datagen_mod, oracle_mod, messi, torch_cuda):
    """Words, leaves and the 100 benchmark queries' answers at 100M x 256,
    all against the oracle (see the module docstring)."""
    torch = torch_cuda
    ix = full["ix"]
    nth = _host_threads()
    pool = concurrent.futures.ThreadPoolExecutor(nth)
    qraw = datagen_mod.random_walks(100, L, seed=datagen_mod.SEED_QUERY, stream=datagen_mod.STREAM_QUERY)
    qz = oracle_mod.znorm(qraw)
    # the GPU side: the benchmark's calls, one query at a time
    _say("full size: 100 benchmark queries, one at a time on the GPU")
    qt = torch.from_numpy(qraw).cuda()
    messi.znorm_(qt)
    np.testing.assert_array_equal(qt.cpu().numpy(), qz)
    gi = np.zeros((100, 1), dtype=np.int64)
    gd = np.zeros((100, 1), dtype=np.float32)
    for i in range(100):
        a, b = ix.knn_plain(qt[i:i + 1].contiguous(), 1)
        gi[i], gd[i] = a.cpu().numpy()[0], b.cpu().numpy()[0]
    words_gpu = ix.export_words()
    # the oracle side, chunk by chunk
    best_d = np.full(100, np.inf)
    best_i = np.full(100, -1, dtype=np.int64)
    owords = np.empty((N, 16), dtype=np.uint8)
    raw_dev = torch.empty((CHUNK, L), dtype=torch.float32, device="cuda")
    t0 = time.time()
    for r0 in range(0, N, CHUNK):
        datagen_mod.gpu_random_walks(raw_dev, row0=r0)  # the seeded generator (not the library)
        raw = raw_dev.cpu().numpy()
        pieces = np.array_split(np.arange(CHUNK), nth)
        zs = list(pool.map(lambda ix_: oracle_mod.znorm(raw[ix_[0]:ix_[-1] + 1]), pieces))
        z = np.concatenate(zs)
        del zs, raw
        ws = list(pool.map(lambda zz: oracle_mod.words(zz, 16, 8), np.array_split(z, nth)))
        owords[r0:r0 + CHUNK] = np.concatenate(ws)
        np.testing.assert_array_equal(words_gpu[r0:r0 + CHUNK], owords[r0:r0 + CHUNK])
        bi, bd, _ = oracle_mod.knn_brute(z, qz, 1, nthreads=nth, row_offset=r0)
        better = (bd[:, 0] < best_d) | ((bd[:, 0] == best_d) & (bi[:, 0] < best_i))
        best_d = np.where(better, bd[:, 0], best_d)
        best_i = np.where(better, bi[:, 0], best_i)
        del z
        _say("  oracle rows %d..%d: words equal, brute force merged (%.0f s)" % (r0, r0 + CHUNK, time.time() - t0))
    del raw_dev
    pool.shutdown()
    np.testing.assert_array_equal(gi[:, 0], best_i)
    np.testing.assert_array_equal(gd[:, 0], np.sqrt(best_d).astype(np.float32))
    _say("full size: 100 answers equal the oracle's brute force; partitioning 100M words on the host")
    oleaves, opos = oracle_mod.build_leaves(owords, 8, 2000)
    del owords
    gleaves, gpos = ix.export_leaves()
    assert len(gleaves) == len(oleaves)
    np.testing.assert_array_equal(gleaves.view(np.uint8), oleaves.view(np.uint8))
    np.testing.assert_array_equal(gpos, opos)
    _say("full size: %d leaves and the position array equal the oracle's (%.0f s)" % (len(oleaves),
                                                                                   time.time() - t0))
