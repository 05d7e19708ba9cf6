"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every oracle function is checked here against something other than itself:
the paper's worked word, published normal quantiles and an independent
quantile routine, closed forms of the mean, invariants of the index, the
iSAX lower-bound inequality, hand-worked examples and brute force.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.special import ndtri

from conftest import golden_path


# ----------------------------------------------------------------------------
# breakpoints
# ----------------------------------------------------------------------------

def test_breakpoints_published_quantiles(oracle_mod):
    rows = [l.split() for l in open(golden_path("normal_quantiles.txt")) if l.strip() and not l.startswith("#")]
    bp8 = oracle_mod.breakpoints(8)
    for p_s, v_s in rows:
        p, v = float(p_s), float(v_s)
        j = int(round(p * 256))
        assert bp8[j - 1] == np.float32(v), (p, bp8[j - 1], v)


@pytest.mark.parametrize("b", range(1, 9))
def test_breakpoints_match_independent_quantile(oracle_mod, b):
    # scipy's ndtri (Cephes rational approximations) is an independent method.
    bp = oracle_mod.breakpoints(b)
    a = 1 << b
    ref = ndtri(np.arange(1, a) / a).astype(np.float32)
    np.testing.assert_array_equal(bp, ref)


def test_breakpoints_structure(oracle_mod):
    bp = oracle_mod.breakpoints(8)
    assert bp.size == 255
    assert np.all(np.diff(bp) > 0)                     # strictly increasing
    assert bp[127] == 0.0                              # median
    np.testing.assert_array_equal(bp[::-1], -bp)       # symmetric
    for c in range(1, 8):                              # nesting of cardinalities
        np.testing.assert_array_equal(oracle_mod.breakpoints(c), bp[(1 << (8 - c)) - 1::1 << (8 - c)])


# ----------------------------------------------------------------------------
# z-normalisation
# ----------------------------------------------------------------------------

def test_znorm_closed_form(oracle_mod, datagen_mod):
    x = datagen_mod.random_walks(2000, 256, seed=3)
    z = oracle_mod.znorm(x).astype(np.float64)
    # mean 0 and population sd 1 (Preliminaries), within fp32 rounding of z
    assert np.max(np.abs(z.sum(1))) < 256 * 16 * 2 ** -23
    assert np.max(np.abs((z * z).sum(1) - 256.0)) < 256 * 2 * 2 ** -22 * 16
    # elementwise against numpy's fp64 mean / std
    xd = x.astype(np.float64)
    ref = (xd - xd.mean(1, keepdims=True)) / xd.std(1, keepdims=True)
    np.testing.assert_allclose(z, ref, rtol=0, atol=2e-6)


def test_znorm_degenerate_and_invariance(oracle_mod):
    x = np.full((3, 64), 7.25, dtype=np.float32)
    x[1] = -3.0
    x[2] = 0.0
    assert np.all(oracle_mod.znorm(x) == 0.0)
    rng = np.random.default_rng(0)
    y = rng.standard_normal((50, 128)).astype(np.float32)
    z1 = oracle_mod.znorm(y)
    z2 = oracle_mod.znorm((4.0 * y + 3.0).astype(np.float32))
    np.testing.assert_allclose(z1, z2, atol=1e-5)


def test_fold_halving_order(oracle_mod):
    # The pinned summation order: pairs (i, i + P/2) first.  For the segment
    # [2^25, 1, -2^25, 1] the fold-halving sum is (2^25 - 2^25) + (1 + 1) = 2,
    # while a left-to-right fp32 sum would give ((2^25 + 1) - 2^25) + 1 = 1.
    seg = np.array([[2.0 ** 25, 1.0, -(2.0 ** 25), 1.0]], dtype=np.float32)
    assert oracle_mod.paa(seg, 1)[0, 0] == np.float32(0.5)


# ----------------------------------------------------------------------------
# PAA
# ----------------------------------------------------------------------------

def test_paa_closed_forms(oracle_mod):
    # piecewise constant -> exact segment values
    vals = np.array([0.5, -1.25, 3.0, 0.0], dtype=np.float32)
    x = np.repeat(vals, 16)[None, :]
    np.testing.assert_array_equal(oracle_mod.paa(x, 4)[0], vals)
    # linear ramp -> centre of each segment, exactly
    ramp = np.arange(256, dtype=np.float32)[None, :]
    want = (np.arange(16) * 16 + 7.5).astype(np.float32)
    np.testing.assert_array_equal(oracle_mod.paa(ramp, 16)[0], want)
    # non power-of-two segment length m = 6 (padded sums, one division)
    ramp6 = np.arange(24, dtype=np.float32)[None, :]
    np.testing.assert_array_equal(oracle_mod.paa(ramp6, 4)[0], np.array([2.5, 8.5, 14.5, 20.5], np.float32))


def test_paa_error_bound(oracle_mod, datagen_mod):
    z = oracle_mod.znorm(datagen_mod.random_walks(3000, 256, seed=4))
    p = oracle_mod.paa(z, 16).astype(np.float64)
    exact = z.astype(np.float64).reshape(3000, 16, 16).mean(2)
    bound = (4 + 1) * 2.0 ** -24 * np.abs(z.astype(np.float64)).reshape(3000, 16, 16).max(2)
    assert np.all(np.abs(p - exact) <= bound)
    # sum of segment means times m is the sum of the series (within the bound)
    assert np.max(np.abs(p.sum(1) * 16 - z.astype(np.float64).sum(1))) < 1e-3


# ----------------------------------------------------------------------------
# symbols, words, root keys
# ----------------------------------------------------------------------------

def test_paper_worked_word(oracle_mod):
    rows = [l for l in open(golden_path("fig1_word.txt")) if l.strip() and not l.startswith("#")]
    for line in rows:
        b_s, paa_s, sym_s, bits_s = [f.strip() for f in line.split("|")]
        b = int(b_s)
        paa = np.array([[float(v) for v in paa_s.split()]], dtype=np.float32)
        sym = oracle_mod.symbols(paa, b)[0]
        assert list(sym) == [int(v) for v in sym_s.split()]
        assert " ".join(format(int(s), "0%db" % b) for s in sym) == bits_s


def test_symbol_tie_rule_and_monotone(oracle_mod):
    bp = oracle_mod.breakpoints(8)
    at = bp[None, :]
    below = np.nextafter(bp, np.float32(-np.inf))[None, :]
    above = np.nextafter(bp, np.float32(np.inf))[None, :]
    j = np.arange(1, 256)
    np.testing.assert_array_equal(oracle_mod.symbols(at.reshape(-1, 1), 8)[:, 0], j)      # on a breakpoint: upper
    np.testing.assert_array_equal(oracle_mod.symbols(below.reshape(-1, 1), 8)[:, 0], j - 1)
    np.testing.assert_array_equal(oracle_mod.symbols(above.reshape(-1, 1), 8)[:, 0], j)
    xs = np.linspace(-4, 4, 5001, dtype=np.float32)[:, None]
    s = oracle_mod.symbols(xs, 8)[:, 0].astype(int)
    assert np.all(np.diff(s) >= 0) and s[0] == 0 and s[-1] == 255


def test_symbol_nesting(oracle_mod, datagen_mod):
    z = oracle_mod.znorm(datagen_mod.random_walks(500, 128, seed=6))
    p = oracle_mod.paa(z, 16)
    s8 = oracle_mod.symbols(p, 8)
    for c in range(1, 8):
        np.testing.assert_array_equal(oracle_mod.symbols(p, c), s8 >> (8 - c))


def test_root_key_bit_order(oracle_mod):
    w = np.array([[128, 0, 255, 127], [0, 0, 0, 200]], dtype=np.uint8)
    assert list(oracle_mod.root_keys(w, 8)) == [0b1010, 0b0001]
    w2 = np.array([[2, 0, 3]], dtype=np.uint8)  # the worked word at 2 bits
    assert list(oracle_mod.root_keys(w2, 2)) == [0b101]


# ----------------------------------------------------------------------------
# leaf partition
# ----------------------------------------------------------------------------

def _read_partition_example():
    d = {}
    leaves = []
    for line in open(golden_path("partition_example.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        key, rest = line.split(None, 1)
        if key == "leaf":
            c, p, sc = [f.split() for f in rest.split("|")]
            leaves.append(([int(v) for v in c], [int(v) for v in p], int(sc[0]), int(sc[1])))
        elif key == "words":
            d["words"] = np.array([[int(v) for v in g.split()] for g in rest.split(";")], dtype=np.uint8)
        elif key == "pos":
            d["pos"] = [int(v) for v in rest.split()]
        else:
            d[key] = int(rest)
    d["leaves"] = leaves
    return d


def test_partition_hand_example(oracle_mod):
    ex = _read_partition_example()
    leaves, pos = oracle_mod.build_leaves(ex["words"], ex["b"], ex["cap"])
    got = [(list(l["card"][:ex["w"]]), list(l["prefix"][:ex["w"]]), int(l["start"]), int(l["count"])) for l in leaves]
    assert got == ex["leaves"]
    assert list(pos) == ex["pos"]


def check_partition(words, b, cap, leaves, pos):
    """Invariants every leaf partition must satisfy (whatever the split rule)."""
    n, w = words.shape
    assert sorted(pos.tolist()) == list(range(n))                       # a partition of the series
    starts = leaves["start"].astype(np.int64)
    counts = leaves["count"].astype(np.int64)
    assert starts[0] == 0 and np.all(starts[1:] == starts[:-1] + counts[:-1]) and counts.sum() == n
    assert np.all(counts >= 1)
    keys = []
    for lf in leaves:
        mem = pos[lf["start"]:lf["start"] + lf["count"]]
        assert np.all(np.diff(mem.astype(np.int64)) > 0)                 # ascending index
        card = lf["card"][:w].astype(int)
        pre = lf["prefix"][:w].astype(int)
        assert np.all(card >= 1) and np.all(card <= b)
        for i in range(w):                                               # members match the node word
            assert np.all((words[mem, i].astype(int) >> (b - card[i])) == pre[i])
        if lf["count"] > cap:                                            # overflow leaf: fully refined
            assert np.all(card == b)
            assert np.all(words[mem] == words[mem[0]])
        # depth-first key: the node's bits, as a path of (prefix bit strings)
        keys.append(tuple((pre[i] << (b - card[i])) for i in range(w)))
    return keys


def _py_partition(words, b, cap):
    """Independent recursive statement of the split rule for tiny inputs."""
    n, w = words.shape
    out = []

    def rec(card, pre, mem):
        if len(mem) <= cap:
            out.append((tuple(card), tuple(pre), list(mem)))
            return
        best, gap = None, None
        for i in range(w):
            if card[i] == b:
                continue
            ones = sum((int(words[x, i]) >> (b - 1 - card[i])) & 1 for x in mem)
            g = abs((len(mem) - ones) - ones)
            if best is None or g < gap:
                best, gap = i, g
        if best is None:
            out.append((tuple(card), tuple(pre), list(mem)))
            return
        for bit in (0, 1):
            sub = [x for x in mem if ((int(words[x, best]) >> (b - 1 - card[best])) & 1) == bit]
            if sub:
                c2, p2 = list(card), list(pre)
                c2[best] += 1
                p2[best] = pre[best] * 2 + bit
                rec(c2, p2, sub)

    keys = {}
    for x in range(n):
        k = tuple((int(words[x, i]) >> (b - 1)) & 1 for i in range(w))
        keys.setdefault(k, []).append(x)
    for k in sorted(keys):
        rec([1] * w, list(k), keys[k])
    return out


@pytest.mark.parametrize("seed", range(40))
def test_partition_tiny_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 13))
    w = int(rng.integers(1, 5))
    b = int(rng.integers(1, 4))
    cap = int(rng.integers(1, 4))
    # few distinct symbols so that duplicates and overflow leaves occur
    words = rng.integers(0, 1 << b, size=(n, w)).astype(np.uint8)
    if seed % 5 == 0:
        words[:] = words[0]
    leaves, pos = oracle_mod.build_leaves(words, b, cap)
    check_partition(words, b, cap, leaves, pos)
    want = _py_partition(words, b, cap)
    got = [(tuple(int(v) for v in l["card"][:w]), tuple(int(v) for v in l["prefix"][:w]),
            pos[l["start"]:l["start"] + l["count"]].tolist()) for l in leaves]
    assert got == want


def test_partition_special_cases(oracle_mod, datagen_mod):
    z = oracle_mod.znorm(datagen_mod.random_walks(3000, 64, seed=8))
    w8 = oracle_mod.words(z, 8, 8)
    keys = oracle_mod.root_keys(w8, 8)
    # capacity >= n: leaves are exactly the non-empty root buckets
    leaves, pos = oracle_mod.build_leaves(w8, 8, 3000)
    uk = np.unique(keys)
    assert len(leaves) == len(uk)
    for lf, k in zip(leaves, uk):
        assert np.all(keys[pos[lf["start"]:lf["start"] + lf["count"]]] == k)
    # one bit per symbol: nothing can split
    w1 = oracle_mod.words(z, 8, 1)
    leaves1, _ = oracle_mod.build_leaves(w1, 1, 5)
    assert len(leaves1) == len(np.unique(oracle_mod.root_keys(w1, 1)))
    assert np.all(leaves1["card"][:, :8] == 1)


def test_partition_invariants_and_split_choice(oracle_mod, datagen_mod):
    n, cap = 20000, 200
    z = oracle_mod.znorm(datagen_mod.random_walks(n, 256, seed=9))
    words = oracle_mod.words(z, 16, 8)
    leaves, pos = oracle_mod.build_leaves(words, 8, cap)
    check_partition(words, 8, cap, leaves, pos)
    # siblings: a leaf and the node next to it that differ in one segment's last
    # bit came from one split; that segment must be the argmin of |n0 - n1| of
    # their union among the parent's refinable segments (ties to the lowest).
    checked = 0
    for a, c in zip(leaves[:-1], leaves[1:]):
        ca, cc = a["card"][:16].astype(int), c["card"][:16].astype(int)
        if not np.array_equal(ca, cc):
            continue
        diff = np.nonzero(a["prefix"][:16] != c["prefix"][:16])[0]
        if len(diff) != 1:
            continue
        s = diff[0]
        if ca[s] < 2:   # root children differ in a card-1 bit; the root is not a balance split
            continue
        if not (a["prefix"][s] % 2 == 0 and c["prefix"][s] == a["prefix"][s] + 1):
            continue
        mem = np.concatenate([pos[a["start"]:a["start"] + a["count"]], pos[c["start"]:c["start"] + c["count"]]])
        pcard = ca.copy()
        pcard[s] -= 1
        gaps = []
        for i in range(16):
            if pcard[i] >= 8:
                gaps.append(None)
                continue
            ones = int(((words[mem, i].astype(int) >> (8 - 1 - pcard[i])) & 1).sum())
            gaps.append(abs(len(mem) - 2 * ones))
        best = min(g for g in gaps if g is not None)
        assert gaps[s] == best and all(g is None or g > best for g in gaps[:s])
        checked += 1
    assert checked > 10


# ----------------------------------------------------------------------------
# lower bound and distances
# ----------------------------------------------------------------------------

def test_d64_definition(oracle_mod):
    q = np.array([1.0, 2.0, 3.0], dtype=np.float32)
    x = np.array([0.5, 4.0, 3.0], dtype=np.float32)
    assert oracle_mod.d64(q, x) == 0.25 + 4.0
    rng = np.random.default_rng(1)
    a, c = rng.standard_normal(256).astype(np.float32), rng.standard_normal(256).astype(np.float32)
    ref = math.fsum((float(u) - float(v)) ** 2 for u, v in zip(a, c))
    assert abs(oracle_mod.d64(a, c) - ref) <= 256 * 2.0 ** -53 * ref


def _d64_variants(q, x):
    """Plausible ways to get D64 wrong, computed with exact rationals and
    correct rounding: a fused multiply-add per term, a pairwise (adjacent)
    tree, and the sequential sum taken backwards."""
    from fractions import Fraction
    d = [float(a) - float(b) for a, b in zip(q.astype(np.float64), x.astype(np.float64))]
    fma = 0.0
    for v in d:
        fma = float(Fraction(fma) + Fraction(v) * Fraction(v))  # one rounding per term
    terms = [v * v for v in d]
    while len(terms) > 1:
        terms = [terms[i] + terms[i + 1] if i + 1 < len(terms) else terms[i] for i in range(0, len(terms), 2)]
    rev = 0.0
    for v in reversed(d):
        rev = rev + v * v
    return {"fma": fma, "pairwise": terms[0], "reversed": rev}


def test_d64_sequential_without_fma(oracle_mod):
    # D64 adds the squared differences in index order, the product and the
    # sum each rounded to fp64.  Worked by hand:
    #   j = 0: d = 128           -> s = 2^14
    #   j = 1: d = 2^-19         -> s = 2^14 + 2^-38 (one unit in the last place at 2^14)
    #   j = 2: d = 1 - 2^-40 (fp32 1 minus fp32 2^-40; exact in fp64)
    #          d^2 = 1 - 2^-39 + 2^-80 rounds to 1 - 2^-39, and
    #          2^14 + 2^-38 + 1 - 2^-39 = 16385 + 2^-39 lies halfway between
    #          16385 (even last bit) and 16385 + 2^-38: ties to even -> 16385.
    # A fused multiply-add keeps the 2^-80 and rounds up to 16385 + 2^-38.
    q = np.array([128.0, 2.0 ** -19, 1.0], dtype=np.float32)
    x = np.array([0.0, 0.0, 2.0 ** -40], dtype=np.float32)
    assert oracle_mod.d64(q, x) == 16385.0
    v = _d64_variants(q, x)
    assert v["fma"] == 16385.0 + 2.0 ** -38
    # the order: 1 followed by 255 terms of 2^-54 (a quarter unit of 1): in
    # index order each rounds away and the sum stays exactly 1; a pairwise
    # tree or the reverse order keeps them (255 * 2^-54 ~ 2^-46)
    q2 = np.concatenate([[1.0], np.full(255, 2.0 ** -27)]).astype(np.float32)
    x2 = np.zeros(256, dtype=np.float32)
    assert oracle_mod.d64(q2, x2) == 1.0
    v2 = _d64_variants(q2, x2)
    assert v2["pairwise"] > 1.0 and v2["reversed"] > 1.0 and v2["fma"] == 1.0


def test_znorm_fold_halving_fp64_order(oracle_mod):
    # z-norm sums in fp64 in fold-halving order.  Worked by hand for
    # x = [2^60, 1, -2^60, 1] (fp32 values, spread beyond fp64's 53 bits):
    #   fold-halving: (2^60 + -2^60) + (1 + 1) = 2 -> mean 0.5
    #   (left to right gives 1 -> 0.25; adjacent pairs give 0 -> 0)
    #   c = x - 0.5 = [2^60, 0.5, -2^60, 0.5] (2^60 - 0.5 rounds to 2^60)
    #   c^2 folded: (2^120 + 2^120) + (0.25 + 0.25) = 2^121 -> variance 2^119
    #   z_1 = fl32(0.5 / 2^59.5) = fl32(2^-60.5), z_0 = fl32(fl64(2^60 / fl64(2^59.5)))
    x = np.array([[2.0 ** 60, 1.0, -(2.0 ** 60), 1.0]], dtype=np.float32)
    z = oracle_mod.znorm(x)[0]
    sigma = math.sqrt(2.0 ** 119)
    assert z[1] == np.float32(0.5 / sigma) and z[3] == z[1]
    assert z[0] == np.float32(2.0 ** 60 / sigma) and z[2] == -z[0]
    # the other orders' means would give c_1 = 0.75 or 1.0 instead
    assert z[1] != np.float32(0.75 / sigma) and z[1] != np.float32(1.0 / sigma)
    # the same within a longer row: zero padding to a power of two (L = 6 -> 8)
    # folds element j onto j + 4: (2^60 + -2^60), (1 + 0), (1 + 0), (0 + 0) -> 2
    y = np.array([[2.0 ** 60, 1.0, 1.0, 0.0, -(2.0 ** 60), 0.0]], dtype=np.float32)
    zy = oracle_mod.znorm(y)[0]
    mean = 2.0 / 6.0
    c = [2.0 ** 60 - mean, 1.0 - mean, 1.0 - mean, -mean, -(2.0 ** 60) - mean, -mean]
    cc = [v * v for v in c] + [0.0, 0.0]
    while len(cc) > 1:
        h = len(cc) // 2
        cc = [cc[i] + cc[i + h] for i in range(h)]
    sig = math.sqrt(cc[0] / 6.0)
    assert zy[1] == np.float32(c[1] / sig) and zy[3] == np.float32(c[3] / sig)


def test_mindist_lower_bounds_ed_all_pairs(oracle_mod, datagen_mod):
    L, w, b = 256, 16, 8
    z = oracle_mod.znorm(datagen_mod.random_walks(1500, L, seed=10))
    q = oracle_mod.znorm(datagen_mod.random_walks(12, L, seed=786, stream=1))
    words = oracle_mod.words(z, w, b)
    # exact (fp64) query PAA; the data words come from fp32 PAA, whose error
    # is covered by widening the regions by the stated slack
    qpaa = q.astype(np.float64).reshape(12, w, L // w).mean(2)
    slack = 6 * 2.0 ** -23 * float(np.abs(z).max())
    full = np.full(w, b)
    for qi in range(12):
        ed = ((z.astype(np.float64) - q[qi].astype(np.float64)) ** 2).sum(1)
        for r in range(0, 1500, 7):
            lb = oracle_mod.mindist_sq(qpaa[qi], full, words[r], b, L // w, slack)
            assert lb <= ed[r] * (1 + 1e-12)
        # the bound of a leaf is below every member's distance
    leaves, pos = oracle_mod.build_leaves(words, b, 50)
    for qi in range(3):
        ed = ((z.astype(np.float64) - q[qi].astype(np.float64)) ** 2).sum(1)
        for lf in leaves:
            lb = oracle_mod.mindist_sq(qpaa[qi], lf["card"][:w], lf["prefix"][:w], b, L // w, slack)
            assert lb <= ed[pos[lf["start"]:lf["start"] + lf["count"]]].min() * (1 + 1e-12)


def test_mindist_special_cases(oracle_mod):
    # m = 1 (w = L): the bound is the squared distance from q to the box
    bp = oracle_mod.breakpoints(2)  # -0.674, 0, 0.674
    q = np.array([-2.0, 0.1, 3.0, 0.3])
    card = np.array([2, 2, 2, 1])
    pre = np.array([1, 2, 2, 1])    # regions [b1,b2]=[-0.67,0], [0,0.67], [0,0.67], [0,inf)
    want = (bp[0] - (-2.0)) ** 2 + 0.0 + (3.0 - bp[2]) ** 2 + 0.0
    assert abs(oracle_mod.mindist_sq(q, card, pre, 2, 1) - want) < 1e-12
    # a query equal to a series: zero against its own word
    rng = np.random.default_rng(2)
    z = oracle_mod.znorm(rng.standard_normal((1, 64)).astype(np.float32))
    p = oracle_mod.paa(z, 8)
    wd = oracle_mod.symbols(p, 8)
    assert oracle_mod.mindist_sq(p[0].astype(np.float64), np.full(8, 8), wd[0], 8, 8) == 0.0


# ----------------------------------------------------------------------------
# exact k-NN
# ----------------------------------------------------------------------------

def _numpy_knn(data, queries, k):
    d = ((queries[:, None, :].astype(np.float64) - data[None, :, :].astype(np.float64)) ** 2).sum(2)
    out = []
    for row in d:
        order = np.lexsort((np.arange(row.size), row))[:k]
        out.append((order, row[order]))
    return out


def test_brute_force_against_numpy(oracle_mod, datagen_mod):
    z = oracle_mod.znorm(datagen_mod.random_walks(3000, 64, seed=12))
    q = oracle_mod.znorm(datagen_mod.random_walks(7, 64, seed=786, stream=1))
    idx, dd, dist = oracle_mod.knn_brute(z, q, 10, nthreads=3)
    for qi, (o, dv) in enumerate(_numpy_knn(z, q, 10)):
        np.testing.assert_array_equal(idx[qi], o)
        np.testing.assert_allclose(dd[qi], dv, rtol=1e-12)
    np.testing.assert_array_equal(dist, np.sqrt(dd).astype(np.float32))


def test_brute_force_all_k_exhaustive(oracle_mod):
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 33, 64):
        data = rng.standard_normal((n, 16)).astype(np.float32)
        q = rng.standard_normal((2, 16)).astype(np.float32)
        ref = _numpy_knn(data, q, n)
        for k in range(1, n + 1):
            idx, dd, _ = oracle_mod.knn_brute(data, q, k, nthreads=2)
            for qi in range(2):
                np.testing.assert_array_equal(idx[qi], ref[qi][0][:k])


def test_ties_go_to_lowest_index(oracle_mod):
    rng = np.random.default_rng(6)
    data = rng.standard_normal((40, 32)).astype(np.float32)
    data[[5, 17, 30]] = data[22]                       # four identical rows
    idx, dd, _ = oracle_mod.knn_brute(data, data[22:23], 3, nthreads=4)
    assert list(idx[0]) == [5, 17, 22] and np.all(dd[0] == 0)


def _isax_vs_brute(oracle_mod, z, q, w, b, cap, k):
    words = oracle_mod.words(z, w, b)
    leaves, pos = oracle_mod.build_leaves(words, b, cap)
    i1, d1, _ = oracle_mod.knn_brute(z, q, k, nthreads=4)
    i2, d2, _ = oracle_mod.knn_isax(z, words, b, leaves, pos, q, k)
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_array_equal(d1, d2)


@pytest.mark.parametrize("k", [1, 5, 40])
def test_isax_search_equals_brute_force(oracle_mod, datagen_mod, k):
    z = oracle_mod.znorm(datagen_mod.random_walks(6000, 128, seed=13))
    q = oracle_mod.znorm(datagen_mod.random_walks(6, 128, seed=786, stream=1))
    qn = datagen_mod.add_noise(z[[3, 999, 4500]], [0.01, 0.1, 1.0])
    _isax_vs_brute(oracle_mod, z, np.concatenate([q, qn]), 16, 8, 100, k)


def test_isax_search_degenerate_inputs(oracle_mod):
    rng = np.random.default_rng(7)
    z = oracle_mod.znorm(rng.standard_normal((500, 32)).astype(np.float32))
    z[100:200] = z[7]                 # a block of duplicates -> ties and overflow leaves
    z[300:310] = 0.0                  # constant series after normalisation
    q = np.concatenate([z[[7, 300, 5]], rng.standard_normal((2, 32)).astype(np.float32)])
    for (w, b, cap, k) in [(8, 8, 10, 1), (8, 8, 10, 30), (4, 1, 3, 5), (16, 3, 1, 2), (1, 8, 1000, 7)]:
        _isax_vs_brute(oracle_mod, z, q, w, b, cap, k)
    # query equal to a dataset row with a lower-index duplicate
    idx, dd, _ = oracle_mod.knn_brute(z, z[150:151], 2)
    assert list(idx[0]) == [7, 100] and np.all(dd[0] == 0)


@pytest.mark.slow
def test_isax_search_tiny_config(oracle_mod, datagen_mod):
    """100,000 random walks of length 256, 16 segments, 8 bits, leaf capacity 2000,
    10 fresh walks as queries, exact 1-NN: the pruned search equals brute force."""
    z = oracle_mod.znorm(datagen_mod.random_walks(100_000, 256))
    q = oracle_mod.znorm(datagen_mod.random_walks(10, 256, seed=datagen_mod.SEED_QUERY,
                                                  stream=datagen_mod.STREAM_QUERY))
    _isax_vs_brute(oracle_mod, z, q, 16, 8, 2000, 1)


# ---------------------------------------------------------------------------
# approximate search (Section 4, approxSearch)
# ---------------------------------------------------------------------------

def test_approx_single_leaf_is_exact(oracle_mod):
    """With one segment and every series above zero the collection falls in a
    single root bucket; with the capacity above N that bucket is the only
    leaf, so the approximate answer is the exact one."""
    rng = np.random.default_rng(3)
    x = (np.abs(rng.standard_normal((900, 8))) + 0.1).astype(np.float32)  # not z-normalised
    q = (np.abs(rng.standard_normal((5, 8))) + 0.1).astype(np.float32)
    words = oracle_mod.words(x, 1, 8)
    leaves, pos = oracle_mod.build_leaves(words, 8, 10_000)
    assert len(leaves) == 1
    for k in (1, 7, 200):
        lf, ia, da, _ = oracle_mod.knn_approx(x, 1, 8, leaves, pos, q, k)
        ib, db, _ = oracle_mod.knn_brute(x, q, k)
        assert np.all(lf == 0)
        np.testing.assert_array_equal(ia, ib)
        np.testing.assert_array_equal(da, db)


def test_approx_picks_the_smallest_bound_and_never_beats_exact(oracle_mod, datagen_mod):
    z = oracle_mod.znorm(datagen_mod.random_walks(8000, 64, seed=21))
    q = np.concatenate([oracle_mod.znorm(datagen_mod.random_walks(6, 64, seed=786, stream=1)),
                        datagen_mod.add_noise(z[[5, 4000]], [0.01, 0.5])]).astype(np.float32)
    words = oracle_mod.words(z, 8, 8)
    leaves, pos = oracle_mod.build_leaves(words, 8, 50)
    for k in (1, 10, 120):
        lf, ia, da, _ = oracle_mod.knn_approx(z, 8, 8, leaves, pos, q, k)
        ib, db, _ = oracle_mod.knn_brute(z, q, k)
        for i in range(len(q)):
            lb = oracle_mod.leaf_bounds(q[i], 8, 8, leaves)
            assert lf[i] == int(np.argmin(lb))                  # first of the smallest
            assert np.all(da[i] >= db[i])                         # the j-th approximate is no better
            # the answers lie in the chosen leaf or, when it holds fewer than
            # k members, in the members that follow it in leaf order
            start, count = int(leaves[lf[i]]["start"]), int(leaves[lf[i]]["count"])
            cnt = min(max(count, k), 4096, len(z))
            r0 = min(start, len(z) - cnt)
            members = set(pos[r0:r0 + cnt].tolist())
            assert set(ia[i].tolist()) <= members
            assert len(set(ia[i].tolist())) == k
    # a dataset row's own leaf has bound 0, and the row is its own answer
    lf, ia, da, _ = oracle_mod.knn_approx(z, 8, 8, leaves, pos, z[[77, 6001]], 1)
    assert list(ia[:, 0]) == [77, 6001] and np.all(da == 0)


# ---- sliding windows of a streaming series (Preliminaries) -----------------

def test_windows_closed_form(oracle_mod):
    """1, 2, ..., 7 in windows of 3: every window is (c - 1, c, c + 1), whose
    z-normalised form is (-sqrt(3/2), 0, sqrt(3/2)) (population sigma
    sqrt(2/3)); with step 2 the windows start at 0, 2, 4, and of 0 .. 7 the
    last value (a tail shorter than a step) starts no window."""
    s = np.arange(1, 8, dtype=np.float32)
    w = oracle_mod.windows(s, 3, 1)
    assert w.shape == (5, 3)
    want = np.array([-np.sqrt(1.5), 0.0, np.sqrt(1.5)], dtype=np.float32)
    np.testing.assert_allclose(w, np.tile(want, (5, 1)), rtol=2e-7, atol=0)
    raw = oracle_mod.windows(s, 3, 2, znorm_windows=False)
    np.testing.assert_array_equal(raw, [[1, 2, 3], [3, 4, 5], [5, 6, 7]])
    raw = oracle_mod.windows(np.arange(8, dtype=np.float32), 3, 2, znorm_windows=False)
    np.testing.assert_array_equal(raw[:, 0], [0, 2, 4])  # the tail value 7 starts no window
    assert oracle_mod.windows(s, 7, 1).shape == (1, 7)


def test_windows_count_and_starts(oracle_mod):
    ramp = np.arange(1000, dtype=np.float32)
    for length, step in ((16, 1), (100, 7), (256, 256), (999, 1), (1000, 3)):
        raw = oracle_mod.windows(ramp, length, step, znorm_windows=False)
        assert raw.shape == ((1000 - length) // step + 1, length)
        np.testing.assert_array_equal(raw[:, 0], np.arange(raw.shape[0]) * step)
        np.testing.assert_array_equal(raw[:, -1] - raw[:, 0], length - 1)


def test_windows_non_overlapping_equal_the_reshaped_collection(oracle_mod, datagen_mod):
    walk = datagen_mod.random_walks(1, 64 * 40, seed=5)[0]
    np.testing.assert_array_equal(oracle_mod.windows(walk, 64, 64), oracle_mod.znorm(walk.reshape(40, 64)))


def test_windows_invariants(oracle_mod, datagen_mod):
    """Each z-normalised window has mean 0 and population variance 1 within
    the rounding of its fp64 statistics; a window is unchanged by an affine
    change of the stream (z-normalisation forgets offset and scale, up to the
    rounding of the scaled values); a constant stretch gives zeros."""
    walk = datagen_mod.random_walks(1, 5000, seed=6)[0].astype(np.float64)
    w = oracle_mod.windows(walk, 128, 3)
    np.testing.assert_allclose(w.astype(np.float64).mean(axis=1), 0.0, atol=1e-5)
    np.testing.assert_allclose(w.astype(np.float64).var(axis=1), 1.0, atol=1e-5)
    w2 = oracle_mod.windows((walk * 4.0 - 1000.0).astype(np.float32), 128, 3)
    np.testing.assert_allclose(w2, w, atol=2e-4)
    s = walk.copy()
    s[2000:2300] = 7.0
    wz = oracle_mod.windows(s, 128, 1)
    assert np.all(wz[2000:2300 - 127] == 0.0) and np.any(wz[1999] != 0.0)
