"""Pins of the oracle's append (Algorithm TreeConstruction's insert and
SplitNode, with the order-free top-down rule): the partition of all series in
which every node that split before splits on the same segment.

  * appending nothing changes nothing; with no split before, an append is a
    plain build of the union;
  * every earlier split is kept, with its segment;
  * a leaf that receives no new series is unchanged (same node, same members);
  * every new leaf lies inside exactly one earlier leaf, or inside a region
    that held no series before; every earlier leaf is the union of the new
    leaves inside it;
  * the new partition keeps the build's invariants (a partition, leaves within
    capacity unless at full cardinality, members ascending, depth-first order),
    and every split that is not an earlier one takes the most balanced
    segment, recomputed by brute force.
"""
import numpy as np
import pytest


def _key(card, prefix, w):
    return bytes(card[:w]) + bytes(prefix[:w])


def _inside(small_card, small_prefix, big_card, big_prefix, w):
    """Region of node `small` inside region of node `big`."""
    for i in range(w):
        if small_card[i] < big_card[i]:
            return False
        if (int(small_prefix[i]) >> (int(small_card[i]) - int(big_card[i]))) != int(big_prefix[i]):
            return False
    return True


def _members(leaves, pos):
    return {_key(l["card"], l["prefix"], 16): pos[l["start"]:l["start"] + l["count"]].tolist() for l in leaves}


def _data(datagen_mod, oracle_mod, n, L, seed):
    return oracle_mod.znorm(datagen_mod.random_walks(n, L, seed=seed))


def _check_partition(oracle_mod, words, leaves, pos, b, cap, w):
    n = len(words)
    assert leaves["count"].sum() == n
    assert np.array_equal(np.sort(pos), np.arange(n))
    starts = leaves["start"].astype(np.int64)
    assert starts[0] == 0 and np.all(starts[1:] == starts[:-1] + leaves["count"][:-1])
    for l in leaves:
        m = pos[l["start"]:l["start"] + l["count"]]
        assert np.all(np.diff(m.astype(np.int64)) > 0)
        for s in range(w):
            assert np.all((words[m, s] >> (b - l["card"][s])) == l["prefix"][s])
        if l["count"] > cap:
            assert np.all(l["card"][:w] == b) and np.all(words[m] == words[m[0]])


def test_append_nothing_and_append_without_earlier_splits(oracle_mod, datagen_mod):
    w, b, cap = 16, 8, 40
    z = _data(datagen_mod, oracle_mod, 3000, 64, 21)
    words = oracle_mod.words(z, w, b)
    l0, p0, inner0 = oracle_mod.build_leaves(words, b, cap, return_inner=True)
    l1, p1, inner1 = oracle_mod.append_leaves(words, b, cap, inner0)
    assert np.array_equal(l0, l1) and np.array_equal(p0, p1) and np.array_equal(inner0, inner1)
    # a capacity no root child exceeds: no splits, so an append is a build of the union
    big = 10 ** 6
    _, _, none = oracle_mod.build_leaves(words[:2000], b, big, return_inner=True)
    assert len(none) == 0
    la, pa, _ = oracle_mod.append_leaves(words, b, big, none)
    lb, pb = oracle_mod.build_leaves(words, b, big)
    assert np.array_equal(la, lb) and np.array_equal(pa, pb)


@pytest.mark.parametrize("n0,n1,cap,L,seed", [(1500, 600, 30, 64, 22), (1200, 1200, 60, 128, 23),
                                              (1500, 100, 10, 32, 24)])
def test_append_keeps_splits_and_is_local(oracle_mod, datagen_mod, n0, n1, cap, L, seed):
    w, b = 16, 8
    z = _data(datagen_mod, oracle_mod, n0 + n1, L, seed)
    words = oracle_mod.words(z, w, b)
    l0, p0, inner0 = oracle_mod.build_leaves(words[:n0], b, cap, return_inner=True)
    l1, p1, inner1 = oracle_mod.append_leaves(words, b, cap, inner0)
    _check_partition(oracle_mod, words, l1, p1, b, cap, w)
    # every earlier split is kept, with its segment
    after = {_key(s["card"], s["prefix"], w): int(s["seg"]) for s in inner1}
    for s in inner0:
        assert after[_key(s["card"], s["prefix"], w)] == int(s["seg"])
    # new leaves refine the earlier ones; untouched leaves are unchanged
    new_members = _members(l1, p1)
    fresh = set(range(n0, n0 + n1))
    for lo in l0:
        inside = [ln for ln in l1 if _inside(ln["card"], ln["prefix"], lo["card"], lo["prefix"], w)]
        got = sorted(x for ln in inside for x in new_members[_key(ln["card"], ln["prefix"], 16)])
        old = p0[lo["start"]:lo["start"] + lo["count"]].tolist()
        assert set(old) <= set(got) and set(got) - set(old) <= fresh
        if set(got) == set(old):  # no new series: the same leaf, the same members
            assert len(inside) == 1 and _key(inside[0]["card"], inside[0]["prefix"], 16) == \
                _key(lo["card"], lo["prefix"], 16) and new_members[_key(lo["card"], lo["prefix"], 16)] == old
    for ln in l1:
        owners = [lo for lo in l0 if _inside(ln["card"], ln["prefix"], lo["card"], lo["prefix"], w)]
        assert len(owners) <= 1
        if not owners:  # a region that held no series: only new ones, and no earlier leaf inside it
            m = new_members[_key(ln["card"], ln["prefix"], 16)]
            assert set(m) <= fresh
            assert not any(_inside(lo["card"], lo["prefix"], ln["card"], ln["prefix"], w) for lo in l0)
    # every split that is not an earlier one is the most balanced
    before = {_key(s["card"], s["prefix"], w) for s in inner0}
    for s in inner1:
        if _key(s["card"], s["prefix"], w) in before:
            continue
        members = [x for ln in l1 if _inside(ln["card"], ln["prefix"], s["card"], s["prefix"], w)
                   for x in new_members[_key(ln["card"], ln["prefix"], 16)]]
        best, best_gap = -1, None
        for i in range(w):
            if s["card"][i] >= b:
                continue
            n_1 = int(np.sum((words[members, i] >> (b - 1 - s["card"][i])) & 1))
            gap = abs(len(members) - 2 * n_1)
            if best < 0 or gap < best_gap:
                best, best_gap = i, gap
        assert int(s["seg"]) == best


def test_append_twice_and_new_regions(oracle_mod, datagen_mod):
    """Two appends in a row, the second with series from regions the first
    index never saw (a different shape of series)."""
    w, b, cap, L = 8, 8, 25, 64
    z = _data(datagen_mod, oracle_mod, 2000, L, 25)
    t = np.linspace(0, 6 * np.pi, L)
    waves = oracle_mod.znorm(np.stack([np.sin(t * (1 + 0.01 * k)) for k in range(300)]).astype(np.float32))
    allz = np.concatenate([z, waves]).astype(np.float32)
    words = oracle_mod.words(allz, w, b)
    l0, p0, i0 = oracle_mod.build_leaves(words[:1200], b, cap, return_inner=True)
    l1, p1, i1 = oracle_mod.append_leaves(words[:2000], b, cap, i0)
    l2, p2, i2 = oracle_mod.append_leaves(words, b, cap, i1)
    _check_partition(oracle_mod, words, l2, p2, b, cap, w)
    keys1 = {_key(s["card"], s["prefix"], w) for s in i1}
    keys2 = {_key(s["card"], s["prefix"], w): int(s["seg"]) for s in i2}
    assert keys1 <= set(keys2)
    assert len(l2) > len(l1)
