"""Pins: decode(encode(volume)) at LOD t equals level L_t of the pyramid,
computed straight from its definition (Sec. 3.1, Alg. 1, Alg. 2)."""
import numpy as np
import pytest

import synth
from brute import pyramid_dense


def bricks_of(vol, b=32):
    nz, ny, nx = vol.shape
    nbx, nby, nbz = nx // b, ny // b, nz // b
    for bid in range(nbx * nby * nbz):
        bx, by, bz = bid % nbx, (bid // nbx) % nby, bid // (nbx * nby)
        yield bid, vol[bz * b:(bz + 1) * b, by * b:(by + 1) * b, bx * b:(bx + 1) * b]


def test_config1_every_brick_every_lod(orc):
    vol = synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1)
    assert (vol == 0).mean() >= 0.30
    blob = orc.encode_volume(vol)
    for bid, br in bricks_of(vol):
        levels, _ = pyramid_dense(br)
        for t in range(6):
            np.testing.assert_array_equal(orc.decode_brick(blob, bid, t), levels[t])


@pytest.mark.parametrize("lane_k", [1, 64, 100000])
@pytest.mark.parametrize("scale_bits", [8, 11, 12])
def test_random_bricks_round_trip(orc, lane_k, scale_bits):
    rng = np.random.default_rng(lane_k + scale_bits)
    vol = np.zeros((32, 32, 64), np.uint32)
    vol[:, :, :32] = synth.random_brick(32, 6, int(rng.integers(1 << 30)), smooth=6)
    vol[:, :, 32:] = synth.random_brick(32, 300, int(rng.integers(1 << 30)), smooth=1)
    blob = orc.encode_volume(vol, lane_k=lane_k, scale_bits=scale_bits)
    for bid, br in bricks_of(vol):
        levels, _ = pyramid_dense(br)
        for t in (0, 1, 2, 5):
            np.testing.assert_array_equal(orc.decode_brick(blob, bid, t), levels[t])


@pytest.mark.parametrize("b", [2, 4, 8, 16, 64])
def test_other_brick_sizes(orc, b):
    vol = synth.voronoi_bg(n=64, sites=40, bg=0.2, seed=b)
    blob = orc.encode_volume(vol, brick_log2=b.bit_length() - 1)
    ids = list(range(0, (64 // b) ** 3, max(1, (64 // b) ** 3 // 7)))
    nb = 64 // b
    for bid in ids:
        bx, by, bz = bid % nb, (bid // nb) % nb, bid // (nb * nb)
        br = vol[bz * b:(bz + 1) * b, by * b:(by + 1) * b, bx * b:(bx + 1) * b]
        levels, _ = pyramid_dense(br)
        for t in range(len(levels)):
            np.testing.assert_array_equal(orc.decode_brick(blob, bid, t), levels[t])


def test_padding_with_zero(orc):
    vol = synth.voronoi_bg(n=64, sites=30, bg=0.0, seed=3)[:40, :50, :33]
    blob = orc.encode_volume(np.ascontiguousarray(vol))
    info = orc.volume_info(blob)
    assert (info["nbx"], info["nby"], info["nbz"]) == (2, 2, 2)
    full = np.zeros((64, 64, 64), np.uint32)
    full[:40, :50, :33] = vol
    for bid, br in bricks_of(full):
        np.testing.assert_array_equal(orc.decode_brick(blob, bid, 0), br)


def test_batch_decode_packs_in_request_order(orc):
    vol = synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1)
    blob = orc.encode_volume(vol)
    ids = [3, 0, 7, 3, 5]
    lods = [0, 2, 1, 5, 3]
    out = orc.decode_bricks(blob, ids, lods)
    o = 0
    for i, t in zip(ids, lods):
        n = (32 >> t) ** 3
        np.testing.assert_array_equal(out[o:o + n], orc.decode_brick(blob, i, t).ravel())
        o += n
    assert o == len(out)


def test_corrupt_record_is_detected(orc):
    # a planted bit flip inside a record's word stream must be reported by the
    # end-of-stream checks (all states back at 2^16, every word consumed)
    vol = synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1)
    blob = orc.encode_volume(vol)
    info = orc.volume_info(blob)
    B, N = info["n_bricks"], info["brick_log2"]
    idx = np.frombuffer(blob, np.uint64, B + 1, 128)
    rs = (128 + 8 * (B + 1) + 15) & ~15
    for bid in range(B):
        w = np.frombuffer(blob, np.uint32, 3 + N, rs + int(idx[bid]))
        P, W, nw = int(w[0]), int(w[1]), int(w[2])
        if nw == 0:
            continue
        words_at = rs + int(idx[bid]) + 4 * (3 + N + P + W)
        for which in (0, nw // 2, nw - 1):
            bad = bytearray(blob)
            bad[words_at + 2 * which] ^= 0x10
            with pytest.raises(orc.OracleError):
                orc.decode_brick(bytes(bad), bid, 0)


@pytest.mark.slow
def test_config2_sampled_bricks(orc):
    vol = synth.cells(n=512, grid=37, seed=2)
    blob = orc.encode_volume(vol)
    nb = 16
    for bid in [0, 1, 17, 273, 1000, 2047, 4095]:
        bx, by, bz = bid % nb, (bid // nb) % nb, bid // (nb * nb)
        br = vol[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32]
        levels, _ = pyramid_dense(br)
        for t in (0, 1, 2):
            np.testing.assert_array_equal(orc.decode_brick(blob, bid, t), levels[t])
