"""messi_knn_noalloc, the search entry point that allocates nothing: its
answers equal those of messi_knn_ex in FP32 mode (the same kernels over
buffers in the library's static device array) bit for bit, and the oracle's
brute force (indices exact, distances fl32 of the fp64 ones), on calls in a
row that shrink, at k = 1 and k > 1; a call that needs more than the array
holds is refused before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N, L = 100_000, 256


@pytest.fixture(scope="module")
def setup(datagen_mod, oracle_mod):
    import torch

    from paper_2009_00786_amd import messi
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    messi.load()
    x = datagen_mod.random_walks(N, L)
    z = oracle_mod.znorm(x)
    fresh = oracle_mod.znorm(datagen_mod.random_walks(8, L, seed=datagen_mod.SEED_QUERY,
                                                      stream=datagen_mod.STREAM_QUERY, row0=900))
    rows = datagen_mod.uniform_ints(8, N, 91, 5)
    noisy = datagen_mod.add_noise(z[rows], np.array([0.01, 0.1, 1.0, 0.1, 0.01, 1.0, 0.1, 0.01]), row0=900)
    q = np.concatenate([fresh, noisy.astype(np.float32)], axis=0)
    xt = torch.from_numpy(z).cuda()
    ix = messi.Index(xt, 16, 8, 2000)
    yield {"ix": ix, "z": z, "q": q, "torch": torch, "messi": messi}
    ix.close()


def _noalloc(s, q, k):
    torch = s["torch"]
    qt = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    oi = torch.full((len(q), k), -7, dtype=torch.int64, device="cuda")
    od = torch.full((len(q), k), -7.0, dtype=torch.float32, device="cuda")
    s["ix"].knn_noalloc(qt, k, out=(oi, od))
    return qt, oi.cpu().numpy(), od.cpu().numpy()


def test_noalloc_equals_knn_ex_and_oracle(setup, oracle_mod):
    s = setup
    torch = s["torch"]
    # two calls in a row, the second smaller (fewer queries, smaller k); then one query at k = 1
    for nq, k in [(16, 10), (3, 4), (1, 1)]:
        q = s["q"][:nq]
        qt, gi, gd = _noalloc(s, q, k)
        ri, rd = s["ix"].knn(qt, k, mode=s["messi"].MODE_FP32)
        np.testing.assert_array_equal(gi, ri.cpu().numpy())
        np.testing.assert_array_equal(gd.view(np.uint32), rd.cpu().numpy().view(np.uint32))
        oi, od, _ = oracle_mod.knn_brute(s["z"], q, k, nthreads=8)
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_array_equal(gd, np.sqrt(od).astype(np.float32))
        torch.cuda.synchronize()


def test_noalloc_allocates_nothing(setup):
    s = setup
    torch = s["torch"]
    q = s["q"]
    _noalloc(s, q[:4], 3)  # first call: the array's address is looked up, the runtime warmed up
    qt = torch.from_numpy(q).cuda()
    oi = torch.empty((len(q), 5), dtype=torch.int64, device="cuda")
    od = torch.empty((len(q), 5), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    s["ix"].knn_noalloc(qt, 5, out=(oi, od))
    s["ix"].knn_noalloc(qt[:2].contiguous(), 5, out=(oi[:2], od[:2]))
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)


def test_noalloc_refuses_beyond_the_array(setup):
    s = setup
    torch = s["torch"]
    messi = s["messi"]
    # 600 queries need about 600 x (128 KiB of candidates + 24 B per leaf) > 64 MiB
    nq = 600
    qt = torch.from_numpy(np.tile(s["q"], (nq // len(s["q"]) + 1, 1))[:nq].copy()).cuda()
    oi = torch.empty((nq, 2), dtype=torch.int64, device="cuda")
    od = torch.empty((nq, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(messi.MessiError) as e:
        s["ix"].knn_noalloc(qt, 2, out=(oi, od))
    assert e.value.code == messi.MESSI_ENOMEM
    # bad arguments are rejected as by messi_knn_ex
    with pytest.raises(messi.MessiError) as e:
        s["ix"].knn_noalloc(qt[:1].contiguous(), 0, out=(oi[:1], od[:1]))
    assert e.value.code == messi.MESSI_EINVAL
    # the array is still usable afterwards
    _, gi, _ = _noalloc(s, s["q"][8:9], 1)
    ri, _ = s["ix"].knn(torch.from_numpy(s["q"][8:9].copy()).cuda(), 1)
    np.testing.assert_array_equal(gi, ri.cpu().numpy())
