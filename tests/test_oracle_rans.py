"""Pins for the oracle's rANS coder (Sec. 3.3): closed form for a uniform
table, state invariants, an information bound, exact round trips."""
import math

import numpy as np
import pytest

L = 1 << 16


@pytest.mark.parametrize("scale_bits", [11, 12])
@pytest.mark.parametrize("W", [1, 2, 8, 64])
def test_uniform_table_closed_form(orc, W, scale_bits):
    # all 16 symbols with frequency M/16: every symbol is exactly 4 bits, a
    # state grows by 4 bits per symbol and sheds 16 bits every 4th symbol
    M = 1 << scale_bits
    f = np.full((2, 16), M // 16, np.uint32)
    rng = np.random.default_rng(W)
    n = 1000 + W
    sym = rng.integers(0, 16, n).astype(np.uint8)
    st, words = orc.rans_encode(sym, f, scale_bits, W)
    per_lane = [len(range(j, n, W)) for j in range(W)]
    assert len(words) == sum(c // 4 for c in per_lane)
    # after c % 4 symbols a state holds 16 + 4 * (c % 4) payload bits above the initial 1
    for j in range(W):
        assert int(st[j]).bit_length() == 17 + 4 * (per_lane[j] % 4)
    out, fin, cur = orc.rans_decode(st, words, n, f, scale_bits)
    np.testing.assert_array_equal(out, sym)
    assert cur == len(words) and (fin == L).all()


def random_tables(rng, scale_bits):
    f = np.zeros((2, 16), np.uint32)
    for t in range(2):
        p = rng.dirichlet(np.full(16, 0.3))
        f[t] = np_normalize(p, 1 << scale_bits)
    return f


def np_normalize(p, M):
    f = np.maximum(1, np.floor(p * M)).astype(np.int64)
    while f.sum() > M:
        f[np.argmax(f)] -= 1
    f[np.argmax(f)] += M - f.sum()
    return f.astype(np.uint32)


@pytest.mark.parametrize("W", [1, 4, 64])
@pytest.mark.parametrize("seed", range(3))
def test_round_trip_and_invariants(orc, W, seed):
    rng = np.random.default_rng(seed * 10 + W)
    S = 11
    f = random_tables(rng, S)
    n = int(rng.integers(1, 5000))
    split = int(rng.integers(0, n + 1))
    p0, p1 = f[0] / f[0].sum(), f[1] / f[1].sum()
    sym = np.concatenate([rng.choice(16, split, p=p0), rng.choice(16, n - split, p=p1)]).astype(np.uint8)
    st, words = orc.rans_encode(sym, f, S, W, tab_split=split)
    assert ((st >= L) & (st < (1 << 32))).all()
    out, fin, cur = orc.rans_decode(st, words, n, f, S, tab_split=split)
    np.testing.assert_array_equal(out, sym)
    assert cur == len(words)
    assert (fin == L).all()
    # information bound: each symbol costs at most log2(M/f) + log2(1 + 2^(S-16)) bits
    M = 1 << S
    info = sum(math.log2(M / f[0 if i < split else 1][s]) for i, s in enumerate(sym))
    spent = 16 * len(words) + sum(math.log2(int(x)) for x in st) - 16 * W
    assert spent <= info + n * math.log2(1 + 2 ** (S - 16)) + 1e-6
    # and it cannot beat the model's information content by more than the
    # rounding slack of the encode step and of each renormalisation
    eps = 2.0 ** (S - 16)
    assert spent >= info - n * (math.log2(1 / (1 - eps)) + math.log2(1 + eps)) - 1e-6


def test_prefix_decode(orc):
    # decoding only the first k symbols needs only a prefix of the words
    rng = np.random.default_rng(5)
    f = random_tables(rng, 11)
    sym = rng.choice(16, 3000, p=f[0] / f[0].sum()).astype(np.uint8)
    st, words = orc.rans_encode(sym, f, 11, 16)
    for k in [0, 1, 17, 1000, 2999]:
        out, _, cur = orc.rans_decode(st, words[:], k, f, 11)
        np.testing.assert_array_equal(out, sym[:k])
        out2, _, cur2 = orc.rans_decode(st, words[:cur], k, f, 11)
        np.testing.assert_array_equal(out2, sym[:k])


def test_wrong_table_breaks_round_trip(orc):
    # a planted mistake (decoding with a different table) must be caught
    rng = np.random.default_rng(9)
    f = random_tables(rng, 11)
    g = f[:, ::-1].copy()
    sym = rng.choice(16, 2000, p=f[0] / f[0].sum()).astype(np.uint8)
    st, words = orc.rans_encode(sym, f, 11, 8)
    try:
        out, fin, cur = orc.rans_decode(st, words, 2000, g, 11)
        assert not ((out == sym).all() and (fin == L).all() and cur == len(words))
    except orc.OracleError:
        pass
