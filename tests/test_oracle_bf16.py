"""Pins of the oracle's BF16 filter model (the batched search's rounding bound).

The bound E on |f - D| is a derivation, not a value the paper prints, so it is
pinned empirically and by construction:
  * each of its two leading parts is approached to within about 1% by a
    constructed pair (every operand rounding aligned; a round-toward-zero
    accumulation that loses every small product), so a smaller constant in
    either part fails;
  * over random, noisy, spiky and adversarial pairs at several lengths, the
    filtered value computed in several accumulation orders (sequential,
    reversed, pairwise, blocks of 32, fold-halving) and in round-toward-zero
    stays within E of the exact squared distance;
  * the oracle's filtered value (sequential order) equals an independent
    numpy simulation bit for bit;
  * at the workload shapes (|q|^2 = |x|^2 = L) E is 4.02 for L = 256 and 2.01
    for L = 128.
"""
import numpy as np
import pytest

F32 = np.float32


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _add32(a, b, mode):
    """fp32 a + b, rounded to nearest or toward zero (arrays of fp32)."""
    if mode == "rn":
        return (a + b).astype(F32)
    s, e = _two_sum(a.astype(np.float64), b.astype(np.float64))  # exact sum = s + e
    r = s.astype(F32)
    over = ((r.astype(np.float64) - s) - e)  # r - exact, sign reliable
    pos = (s + e) > 0
    neg = (s + e) < 0
    down = pos & (over > 0)
    up = neg & (over < 0)
    r = np.where(down, np.nextafter(r, F32(0)), r)
    r = np.where(up, np.nextafter(r, F32(0)), r)
    return r.astype(F32)


def _accumulate(p, order, mode):
    """Sum the rows of p (npairs x L, fp32) in the given order."""
    n, L = p.shape
    if order == "seq":
        s = np.zeros(n, F32)
        for j in range(L):
            s = _add32(s, p[:, j], mode)
        return s
    if order == "rev":
        s = np.zeros(n, F32)
        for j in range(L - 1, -1, -1):
            s = _add32(s, p[:, j], mode)
        return s
    if order == "pairwise":
        v = p.copy()
        while v.shape[1] > 1:
            if v.shape[1] % 2:
                v = np.concatenate([v, np.zeros((n, 1), F32)], axis=1)
            v = _add32(v[:, 0::2], v[:, 1::2], mode)
        return v[:, 0]
    if order == "fold":
        P = 1
        while P < L:
            P *= 2
        v = np.concatenate([p, np.zeros((n, P - L), F32)], axis=1)
        while v.shape[1] > 1:
            h = v.shape[1] // 2
            v = _add32(v[:, :h], v[:, h:], mode)
        return v[:, 0]
    if order == "block32":  # 32 products per step, then the running sum
        s = np.zeros(n, F32)
        for j0 in range(0, L, 32):
            blk = np.zeros(n, F32)
            for j in range(j0, min(L, j0 + 32)):
                blk = _add32(blk, p[:, j], mode)
            s = _add32(s, blk, mode)
        return s
    raise ValueError(order)


def _filtered(oracle_mod, q, x, order, mode):
    qb, xb = oracle_mod.bf16_round(q), oracle_mod.bf16_round(x)
    p = (qb * xb).astype(F32)  # exact: 8-bit significands
    s = _accumulate(p, order, mode)
    a2 = np.sum(q.astype(np.float64) ** 2, axis=1)
    b2 = np.sum(x.astype(np.float64) ** 2, axis=1)
    nsum = (a2.astype(F32) + b2.astype(F32)).astype(F32)
    return (nsum - F32(2) * s).astype(F32), a2, b2


def _exact_d(q, x):
    d = q.astype(np.float64) - x.astype(np.float64)
    return np.sum(d * d, axis=1)


def _bounds(oracle_mod, a2, b2, L):
    return np.array([oracle_mod.bf16_error_bound(a, b, L) for a, b in zip(a2, b2)])


def _pairs(datagen_mod, oracle_mod, L, n, seed):
    """Random z-normalised walks against each other, noisy copies, a spike."""
    z = oracle_mod.znorm(datagen_mod.random_walks(2 * n, L, seed=seed))
    q, x = z[:n], z[n:]
    sig = np.array([(0.01, 0.1, 1.0)[i % 3] for i in range(n)])
    xn = datagen_mod.add_noise(q, sig, seed=seed + 1).astype(F32)
    spike = np.zeros((1, L), F32)
    spike[0, L // 3] = np.sqrt(L)
    qs = np.concatenate([q, q, spike, spike * -1], axis=0)
    xs = np.concatenate([x, xn, q[:1], q[1:2]], axis=0)
    return qs.astype(F32), xs.astype(F32)


@pytest.mark.parametrize("L", [256, 128])
def test_bound_at_the_workload_shapes(oracle_mod, L):
    # z-normalised rows: |q|^2 = |x|^2 = L
    e = oracle_mod.bf16_error_bound(L, L, L)
    assert e == pytest.approx(4.02 if L == 256 else 2.01, abs=0.01)


def test_operand_part_is_tight(oracle_mod):
    """Every operand sits just below a BF16 rounding midpoint, so every product
    loses nearly (2 u_b + u_b^2) of its value in the same direction."""
    L = 256
    v = F32(1.0 + 2.0 ** -8 - 2.0 ** -20)
    assert oracle_mod.bf16_round(np.array([v]))[0] == 1.0
    sign = np.where(np.arange(L) % 3 == 0, -1.0, 1.0).astype(F32)
    q = (v * sign)[None, :]
    x = q.copy()
    qb, xb = oracle_mod.bf16_round(q), oracle_mod.bf16_round(x)
    err = abs(np.dot(qb[0].astype(np.float64), xb[0]) - np.dot(q[0].astype(np.float64), x[0]))
    a2 = float(np.sum(q.astype(np.float64) ** 2))
    _, t = oracle_mod.bf16_error_bound(a2, a2, L, terms=True)
    ratio = err / (t[0] / 2)
    assert 0.99 < ratio <= 1.0
    # and the whole bound covers the filtered value, with little to spare
    f, a2v, b2v = _filtered(oracle_mod, q, x, "seq", "rn")
    D = _exact_d(q, x)
    E = oracle_mod.bf16_error_bound(a2v[0], b2v[0], L)
    assert abs(float(f[0]) - D[0]) <= E
    assert abs(float(f[0]) - D[0]) > 0.98 * E


@pytest.mark.parametrize("L", [256, 1024])
def test_accumulation_part_is_tight(oracle_mod, L):
    """One unit product then L - 1 products just below half of ulp(1) squared:
    rounding toward zero drops every one of them, which is the worst case
    the recursive-summation bound gamma_{L-1} allows."""
    eps = F32(1.4140625 * 2.0 ** -12)  # exact in BF16; eps^2 just below 2^-23
    assert oracle_mod.bf16_round(np.array([eps]))[0] == eps
    q = np.full((1, L), eps, F32)
    q[0, 0] = 1.0
    p = (q * q).astype(F32)
    s = _accumulate(p, "seq", "rz")
    assert s[0] == 1.0  # every small product lost
    exact = float(np.sum(p.astype(np.float64)))
    a2 = float(np.sum(q.astype(np.float64) ** 2))
    _, t = oracle_mod.bf16_error_bound(a2, a2, L, terms=True)
    ratio = (exact - float(s[0])) / (t[1] / 2)
    assert 0.99 < ratio <= 1.0


@pytest.mark.parametrize("L", [256, 128, 96])
def test_bound_holds_in_every_order(oracle_mod, datagen_mod, L):
    q, x = _pairs(datagen_mod, oracle_mod, L, 20000, seed=40 + L)
    D = _exact_d(q, x)
    worst = 0.0
    E = None
    for order in ("seq", "rev", "pairwise", "block32", "fold"):
        for mode in ("rn", "rz"):
            f, a2, b2 = _filtered(oracle_mod, q, x, order, mode)
            if E is None:
                E = _bounds(oracle_mod, a2, b2, L)
            r = np.abs(f.astype(np.float64) - D) / E
            worst = max(worst, float(r.max()))
            assert np.all(r < 1.0), (order, mode, float(r.max()))
    assert worst > 0.001  # the pairs do exercise the bound


def test_adversarial_pairs(oracle_mod):
    """Operands at rounding midpoints and just off them, same-sign products,
    long rows, round-toward-zero accumulation."""
    rng = np.random.default_rng(9)
    for L in (32, 256, 1024):
        n = 512
        # significands 1 + (k + 1/2) 2^-7 +- tiny: BF16 rounding midpoints
        k = rng.integers(0, 128, size=(n, L))
        mid = (1.0 + (k + 0.5) * 2.0 ** -7) * 2.0 ** rng.integers(-3, 3, size=(n, L))
        jitter = rng.choice([-1.0, 0.0, 1.0], size=(n, L)) * 2.0 ** -20
        q = (mid * (1.0 + jitter)).astype(F32)
        x = (q * np.where(rng.random((n, L)) < 0.9, 1.0, -1.0)).astype(F32)
        x = (x * (1.0 + 2.0 ** -9 * rng.random((n, L)))).astype(F32)
        D = _exact_d(q, x)
        for order in ("seq", "pairwise"):
            for mode in ("rn", "rz"):
                f, a2, b2 = _filtered(oracle_mod, q, x, order, mode)
                E = _bounds(oracle_mod, a2, b2, L)
                assert np.all(np.abs(f.astype(np.float64) - D) < E), (L, order, mode)


def test_oracle_filter_value_matches_a_plain_simulation(oracle_mod, datagen_mod):
    q, x = _pairs(datagen_mod, oracle_mod, 256, 500, seed=77)
    got = oracle_mod.bf16_filter_values(q, x)
    want, _, _ = _filtered(oracle_mod, q, x, "seq", "rn")
    np.testing.assert_array_equal(got, want)


def test_bf16_rounding_definition(oracle_mod):
    # nearest, ties to even, at the scale of 1: ulp 2^-7
    one = 1.0
    vals = np.array([one, one + 2 ** -8, one + 3 * 2 ** -8, one + 2 ** -8 + 2 ** -20, one + 2 ** -8 - 2 ** -20,
                     -(one + 3 * 2 ** -8), 2.0 ** -130, 65504.0], dtype=F32)
    want = np.array([one, one, one + 2 ** -6, one + 2 ** -7, one, -(one + 2 ** -6), 2.0 ** -130, 65536.0],
                    dtype=F32)
    np.testing.assert_array_equal(oracle_mod.bf16_round(vals), want)
