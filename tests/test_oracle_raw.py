"""Pins of the oracle's coding without rANS (Table 1's "no rANS" variant):
the decoded blocks equal the resolution pyramid's levels, each record holds
exactly its symbol stream packed four nibbles to a 16-bit word, and a
malformed raw record is refused."""
import numpy as np
import pytest

import synth
from brute import pyramid_dense

HDR = 128


def record(blob, bid):
    """(record words as uint32, record bytes) of brick bid."""
    B = int(np.frombuffer(blob, np.uint32, 1, 36)[0])
    idx = np.frombuffer(blob, np.uint64, B + 1, HDR)
    rs = (HDR + 8 * (B + 1) + 15) & ~15
    a, b = rs + int(idx[bid]), rs + int(idx[bid + 1])
    return np.frombuffer(blob, np.uint32, (b - a) // 4, a), blob[a:b]


def bricks(vol, b):
    nz, ny, nx = vol.shape
    for bz in range(nz // b):
        for by in range(ny // b):
            for bx in range(nx // b):
                yield vol[bz * b:(bz + 1) * b, by * b:(by + 1) * b, bx * b:(bx + 1) * b]


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_raw_decode_is_the_pyramid(orc, N):
    b = 1 << N
    n = max(64, b)
    rng = np.random.default_rng(N)
    vol = synth.voronoi_bg(n=n, sites=40 + 10 * N, bg=0.25, seed=N)
    vol[: n // 2, : n // 4, :] = rng.integers(1, 6, size=(n // 2, n // 4, n)).astype(np.uint32)
    blob = orc.encode_volume(vol, brick_log2=N, tables=0)
    assert orc.volume_info(blob)["brick_log2"] == N
    assert int(np.frombuffer(blob, np.uint32, 1, 56)[0]) == 1  # the coding word
    for bid, br in enumerate(bricks(vol, b)):
        if bid % 7:
            continue
        levels, _ = pyramid_dense(br)
        for t in range(N + 1):
            np.testing.assert_array_equal(orc.decode_brick(blob, bid, t), levels[t])


@pytest.mark.parametrize("N", [2, 4, 5])
def test_raw_record_is_the_packed_symbol_stream(orc, N):
    b = 1 << N
    vol = synth.cells(n=64, grid=7, seed=3 + N)
    blob = orc.encode_volume(vol, brick_log2=N, tables=0)
    for bid, br in enumerate(bricks(vol, b)):
        if bid % 5:
            continue
        sym, cum, pal = orc.brick_symbols(br)
        w, raw = record(blob, bid)
        n, P = len(sym), len(pal)
        nw = (n + 3) // 4
        hdr = 3 + N
        # P, no states, the word count, the cumulative counts, the palette
        assert (int(w[0]), int(w[1]), int(w[2])) == (P, 0, nw)
        np.testing.assert_array_equal(w[3:hdr], cum)
        np.testing.assert_array_equal(w[hdr:hdr + P], pal)
        # exactly the symbols, four to a 16-bit word, low nibble first
        want = np.zeros(nw, np.uint16)
        for i, s in enumerate(sym):
            want[i // 4] |= np.uint16(int(s) << (4 * (i % 4)))
        got = np.frombuffer(raw, np.uint16, nw, 4 * (hdr + P))
        np.testing.assert_array_equal(got, want)
        assert len(raw) == (4 * (hdr + P) + 2 * nw + 3) // 4 * 4


def test_raw_and_rans_codings_share_the_symbol_stream(orc):
    vol = synth.cells(n=64, grid=6, seed=9)
    raw = orc.encode_volume(vol, tables=0)
    rans = orc.encode_volume(vol, tables=2)
    for bid in range(8):
        wr, _ = record(raw, bid)
        wa, _ = record(rans, bid)
        # same palette size and cumulative counts; only the coding differs
        assert wr[0] == wa[0]
        np.testing.assert_array_equal(wr[3:8], wa[3:8])
        for t in (0, 2):
            np.testing.assert_array_equal(orc.decode_brick(raw, bid, t), orc.decode_brick(rans, bid, t))


def test_malformed_raw_records_are_refused(orc):
    vol = synth.cells(n=32, grid=5, seed=4)
    blob = bytearray(orc.encode_volume(vol, tables=0))
    w, raw = record(bytes(blob), 0)
    n, P = int(w[3]), int(w[0])
    B = int(np.frombuffer(bytes(blob), np.uint32, 1, 36)[0])
    rs = (HDR + 8 * (B + 1) + 15) & ~15
    off = rs + int(np.frombuffer(bytes(blob), np.uint64, 1, HDR)[0])
    # a state count on a raw record
    bad = bytearray(blob)
    bad[off + 4] = 1
    with pytest.raises(RuntimeError):
        orc.decode_brick(bytes(bad), 0, 0)
    # a set nibble past the last symbol (only when the last word is part-used)
    if n % 4:
        bad = bytearray(blob)
        last = off + 4 * (8 + P) + 2 * ((n + 3) // 4 - 1)
        v = int.from_bytes(bad[last:last + 2], "little") | (1 << (4 * (n % 4)))
        bad[last:last + 2] = v.to_bytes(2, "little")
        with pytest.raises(RuntimeError):
            orc.decode_brick(bytes(bad), 0, 0)
    # an unknown coding
    bad = bytearray(blob)
    bad[56] = 2
    with pytest.raises(RuntimeError):
        orc.decode_brick(bytes(bad), 0, 0)
