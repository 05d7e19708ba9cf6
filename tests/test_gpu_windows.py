"""GPU parity of the windows of a streaming series (the paper's sliding-window
subsequences, Preliminaries): the rows the library writes equal the oracle's
z-normalised windows bit for bit, and an index over them answers k-NN exactly
(window indices as the oracle's brute force over the same windows)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


CASES = [
    # m, len, step, znorm
    (100_000, 256, 1, True),
    (50_003, 100, 3, True),     # padded rows, a ragged tail
    (20_000, 16, 1, True),      # short windows: copied, then z-normalised in place
    (30_000, 1024, 7, True),
    (4_096, 4_096 // 4, 1024, True),
    (256, 256, 1, True),        # one window
    (10_000, 64, 5, False),     # plain copy
    (777, 33, 2, True),
]


@pytest.mark.parametrize("m,length,step,znorm", CASES)
def test_windows_bitwise(torch_cuda, messi, datagen_mod, oracle_mod, m, length, step, znorm):
    _say("windows m=%d len=%d step=%d znorm=%d" % (m, length, step, znorm))
    s = datagen_mod.random_walks(1, m, seed=31)[0]
    got = messi.windows(torch_cuda.from_numpy(s).cuda(), length, step, znorm).cpu().numpy()
    want = oracle_mod.windows(s, length, step, znorm_windows=znorm)
    assert got.shape == want.shape
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


def test_windows_constant_stretch_and_errors(torch_cuda, messi, oracle_mod):
    torch = torch_cuda
    s = np.linspace(-3, 5, 3000).astype(np.float32)
    s[1000:1500] = 2.5
    got = messi.windows(torch.from_numpy(s).cuda(), 200, 1).cpu().numpy()
    np.testing.assert_array_equal(got, oracle_mod.windows(s, 200, 1))
    assert np.all(got[1000:1301] == 0.0)
    t = torch.from_numpy(s).cuda()
    for args in ((t, 3001, 1), (t, 0, 1), (t, 1025, 1), (t, 100, 0)):
        with pytest.raises(messi.MessiError) as e:
            messi.windows(*args)
        assert e.value.code == messi.MESSI_EINVAL
    # output overlapping the input
    buf = torch.zeros(20_000, dtype=torch.float32, device="cuda")
    with pytest.raises(messi.MessiError) as e:
        messi.windows(buf[:1000], 10, 1, out=buf[500:].view(-1, 10)[:991])
    assert e.value.code == messi.MESSI_EINVAL
    # non-finite values are reported with z-normalisation
    bad = torch.from_numpy(s.copy()).cuda()
    bad[1234] = float("nan")
    with pytest.raises(messi.MessiError) as e:
        messi.windows(bad, 64, 1)
    assert e.value.code == messi.MESSI_EINVAL


@pytest.mark.parametrize("k", [1, 10])
def test_windows_index_knn(torch_cuda, messi, datagen_mod, oracle_mod, k):
    torch = torch_cuda
    m, length = 200_000, 256
    _say("windows index m=%d len=%d k=%d" % (m, length, k))
    s = datagen_mod.random_walks(1, m, seed=32)[0]
    rows = messi.windows(torch.from_numpy(s).cuda(), length, 1)
    ix = messi.Index(rows, 16, 8, 2000)
    w = oracle_mod.windows(s, length, 1)
    starts = datagen_mod.uniform_ints(6, len(w), 33, 5)
    noisy = datagen_mod.add_noise(w[starts], [0.0, 0.01, 0.1, 1.0, 0.1, 0.01])
    fresh = oracle_mod.znorm(datagen_mod.random_walks(4, length, seed=datagen_mod.SEED_QUERY,
                                                      stream=datagen_mod.STREAM_QUERY))
    q = np.concatenate([noisy, fresh]).astype(np.float32)
    oidx, od, _ = oracle_mod.knn_brute(w, q, k, nthreads=8)
    for mode in (messi.MODE_FP32,):
        gi, gd = ix.knn(torch.from_numpy(q).cuda(), k, mode=mode)
        np.testing.assert_array_equal(gi.cpu().numpy(), oidx)
        np.testing.assert_array_equal(gd.cpu().numpy(), np.sqrt(od).astype(np.float32))
    assert oidx[0, 0] == starts[0]  # an exact window finds its own start
    ix.close()
