"""GPU parity of appending series to an index (Algorithm TreeConstruction's
insert and SplitNode): after each append the leaves, the member order and the
words equal the oracle's append bit for bit, and k-NN over the grown
collection equals brute force (FP32 and BF16 modes)."""
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


def _same_index(ix, leaves, pos, words, w):
    gl, gp = ix.export_leaves()
    assert len(gl) == len(leaves)
    np.testing.assert_array_equal(gl["card"][:, :w], leaves["card"][:, :w])
    np.testing.assert_array_equal(gl["prefix"][:, :w], leaves["prefix"][:, :w])
    np.testing.assert_array_equal(gl["start"], leaves["start"])
    np.testing.assert_array_equal(gl["count"], leaves["count"])
    np.testing.assert_array_equal(gp, pos)
    np.testing.assert_array_equal(ix.export_words(), words)


@pytest.mark.parametrize("L,w,cap,steps", [(128, 16, 200, (40_000, 50_000, 75_000)),
                                           (64, 8, 25, (3_000, 3_001, 9_000, 9_000)),
                                           (96, 16, 1, (500, 700))])
def test_append_matches_oracle(torch_cuda, messi, datagen_mod, oracle_mod, L, w, cap, steps):
    torch = torch_cuda
    b = 8
    total = steps[-1]
    raw = datagen_mod.random_walks(total, L, seed=61)
    if L == 64:  # the last rows from regions the first index never saw
        t = np.linspace(0, 6 * np.pi, L)
        raw[-1000:] = np.stack([np.sin(t * (1 + 0.003 * k)) for k in range(1000)]).astype(np.float32)
    z = oracle_mod.znorm(raw)
    words = oracle_mod.words(z, w, b)
    dev = torch.from_numpy(z).cuda()
    _say("append L=%d w=%d cap=%d steps=%s" % (L, w, cap, steps))
    ix = messi.Index(dev[:steps[0]].contiguous(), w, b, cap, bf16_shadow=True)
    leaves, pos, inner = oracle_mod.build_leaves(words[:steps[0]], b, cap, return_inner=True)
    _same_index(ix, leaves, pos, words[:steps[0]], w)
    for n in steps[1:]:
        ix.append(dev[:n].contiguous())
        leaves, pos, inner = oracle_mod.append_leaves(words[:n], b, cap, inner)
        _say("  n=%d leaves=%d" % (n, len(leaves)))
        _same_index(ix, leaves, pos, words[:n], w)
        assert ix.info()["n"] == n
    q = np.concatenate([z[[0, total - 1, total // 2]],
                        oracle_mod.znorm(datagen_mod.random_walks(3, L, seed=62))]).astype(np.float32)
    oi, _, od = oracle_mod.knn_brute(z, q, 5, nthreads=8)
    for mode in (messi.MODE_FP32, messi.MODE_BF16):
        gi, gd = ix.knn(torch.from_numpy(q).cuda(), 5, mode=mode)
        np.testing.assert_array_equal(gi.cpu().numpy(), oi)
        np.testing.assert_array_equal(gd.cpu().numpy(), od)
    ix.close()


def test_append_errors_leave_the_index_unchanged(torch_cuda, messi, datagen_mod, oracle_mod):
    torch = torch_cuda
    z = oracle_mod.znorm(datagen_mod.random_walks(3000, 64, seed=63))
    dev = torch.from_numpy(z).cuda()
    ix = messi.Index(dev[:2000].contiguous(), 16, 8, 30)
    before = ix.export_leaves()
    with pytest.raises(messi.MessiError) as e:
        ix.append(dev[:1999].contiguous())  # fewer rows than indexed
    assert e.value.code == messi.MESSI_EINVAL
    bad = dev.clone()
    bad[2500, 7] = float("nan")
    with pytest.raises(messi.MessiError) as e:
        ix.append(bad)
    assert e.value.code == messi.MESSI_EINVAL
    after = ix.export_leaves()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    ix.append(dev[:2000].contiguous())  # nothing new: the same partition
    again = ix.export_leaves()
    assert np.array_equal(before[0], again[0]) and np.array_equal(before[1], again[1])
    ix.close()
