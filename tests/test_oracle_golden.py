"""Pins: the oracle's symbol streams for hand-worked bricks (tests/golden),
and their decode at every level of detail."""
import glob
import json
import os

import numpy as np
import pytest

from brute import pyramid_dense

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FILES = sorted(glob.glob(os.path.join(GOLD, "*.json")))


def make_brick(g):
    b = g["b"]
    L = g["labels"]
    if g["kind"] == "uniform":
        return np.full((b, b, b), L["A"], np.uint32)
    if g["kind"] == "halfspace_x":
        a = np.full((b, b, b), L["B"], np.uint32)
        a[:, :, :g["split"]] = L["A"]
        return a
    if g["kind"] == "checkerboard":
        z, y, x = np.meshgrid(np.arange(b), np.arange(b), np.arange(b), indexing="ij")
        return np.where((x + y + z) % 2 == 0, L["A"], L["B"]).astype(np.uint32)
    if g["kind"] == "points":
        a = np.full((b, b, b), L[g["background"]], np.uint32)
        for x, y, z, c in g["points"]:
            a[z, y, x] = L[c]
        return a
    if g["kind"] == "children":
        a = np.zeros((2, 2, 2), np.uint32)
        for k, c in enumerate(g["children"]):
            a[k >> 2, (k >> 1) & 1, k & 1] = L[c]
        return a
    raise ValueError(g["kind"])


def expand(segments):
    segs = []
    for runs in segments:
        s = []
        for rep, pat in runs:
            s += list(pat) * rep
        segs.append(s)
    return segs


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f) for f in FILES])
def test_golden_brick(orc, path):
    g = json.load(open(path))
    brick = make_brick(g)
    sym, cum, pal = orc.brick_symbols(brick)
    segs = expand(g["segments"])
    N = g["b"].bit_length() - 1
    assert len(segs) == N
    want = [v for s in segs for v in s]
    assert list(sym) == want
    # cum[m] = symbols through the segment of child level m (segments listed coarse to fine)
    acc, want_cum = 0, [0] * N
    for i, s in enumerate(segs):
        acc += len(s)
        want_cum[N - 1 - i] = acc
    assert list(cum) == want_cum
    assert list(pal) == [g["labels"][c] for c in g["palette"]]
    # decoding the stream at every level of detail gives the pyramid level
    levels, _ = pyramid_dense(brick)
    for t in range(N + 1):
        np.testing.assert_array_equal(orc.replay(sym, cum, pal, N, t), levels[t])


def test_checkerboard_has_maximal_symbol_count(orc):
    g = json.load(open(os.path.join(GOLD, "b3_checker32.json")))
    sym, cum, pal = orc.brick_symbols(make_brick(g))
    assert len(sym) == sum(8 ** k for k in range(1, 6)) == 37448
