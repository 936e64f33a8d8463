"""Pins for the two static frequency tables (Sec. 3.3, Sec. 3.4 prepass)."""
import numpy as np
import pytest

import synth


def test_table_closed_forms(orc):
    # no counts: +1 smoothing gives exactly M/16 each
    np.testing.assert_array_equal(orc.normalize_table(np.zeros(16), 11), np.full(16, 128))
    # one dominant symbol: 15 symbols get the floor of 1, the surplus is
    # taken from the largest entry one at a time
    c = np.zeros(16, np.uint64)
    c[15] = 10 ** 6
    want = np.ones(16, np.uint32)
    want[15] = 2048 - 15
    np.testing.assert_array_equal(orc.normalize_table(c, 11), want)
    # three equal counts of 999: floor(1000 * 4096 / 3013) = 1359 each, the
    # others floor(4096 / 3013) = 1; the deficit 4096 - 4090 = 6 goes to the
    # first of the largest entries
    c = np.zeros(16, np.uint64)
    c[:3] = 999
    want = np.ones(16, np.uint32)
    want[:3] = [1365, 1359, 1359]
    np.testing.assert_array_equal(orc.normalize_table(c, 12), want)


@pytest.mark.parametrize("seed", range(5))
def test_table_invariants(orc, seed):
    rng = np.random.default_rng(seed)
    c = rng.integers(0, 10 ** rng.integers(1, 7), 16).astype(np.uint64)
    for S in (8, 11, 12):
        f = orc.normalize_table(c, S)
        assert f.sum() == 1 << S and (f >= 1).all()
        ideal = (c + 1) * (1 << S) / (c + 1).sum()
        assert np.abs(f - ideal).max() <= 16 + 1


def test_tables_recount_from_sampled_bricks(orc):
    # the container's two tables are the normalised nibble counts of every
    # stride-th brick: interior nibbles (children at level >= 1) and leaf ones
    vol = synth.voronoi_bg(n=96, sites=60, seed=21)
    stride = 5
    blob = orc.encode_volume(vol, sample_stride=stride, scale_bits=11)
    info = orc.volume_info(blob)
    nb = info["nbx"]
    cnt = np.zeros((2, 16), np.uint64)
    for bid in range(0, info["n_bricks"], stride):
        bx, by, bz = bid % nb, (bid // nb) % nb, bid // (nb * nb)
        br = np.ascontiguousarray(vol[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32])
        sym, cum, _ = orc.brick_symbols(br)
        split = int(cum[1])
        np.add.at(cnt[0], sym[:split].astype(np.int64), 1)
        np.add.at(cnt[1], sym[split:].astype(np.int64), 1)
    # leaf children never carry a stop bit
    assert cnt[1][8:].sum() == 0
    for t in range(2):
        np.testing.assert_array_equal(info["freq"][t], orc.normalize_table(cnt[t], 11))


def test_one_table_is_the_normalised_sum(orc):
    # Table 1's variant: one frequency table from the counts of all symbols
    # of the sampled bricks, stored in both table slots; lossless as before
    vol = synth.voronoi_bg(n=96, sites=60, seed=21)
    stride = 5
    blob = orc.encode_volume(vol, sample_stride=stride, scale_bits=11, tables=1)
    info = orc.volume_info(blob)
    nb = info["nbx"]
    cnt = np.zeros(16, np.uint64)
    for bid in range(0, info["n_bricks"], stride):
        bx, by, bz = bid % nb, (bid // nb) % nb, bid // (nb * nb)
        br = np.ascontiguousarray(vol[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32])
        sym, _, _ = orc.brick_symbols(br)
        np.add.at(cnt, sym.astype(np.int64), 1)
    want = orc.normalize_table(cnt, 11)
    np.testing.assert_array_equal(info["freq"][0], want)
    np.testing.assert_array_equal(info["freq"][1], want)
    for bid in range(info["n_bricks"]):
        bx, by, bz = bid % nb, (bid // nb) % nb, bid // (nb * nb)
        np.testing.assert_array_equal(orc.decode_brick(blob, bid, 0),
                                      vol[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32])
