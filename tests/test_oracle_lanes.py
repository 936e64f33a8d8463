"""The interleaving width of every record follows the format's lane rule.

The rule is this project's choice (the paper codes each brick as one rANS
stream): a brick with n > 0 symbols gets W = the largest power of two that
is at most min(lane_max, n / lane_k), and at least 1; a brick without
symbols gets W = 0.  Here it is evaluated as min(lane_max, 2^floor(log2(n //
lane_k))) from each record's own symbol count, for every record of volumes
encoded by the oracle under several parameters.
"""
import numpy as np
import pytest

import synth


def records(blob):
    nb = int(np.frombuffer(blob, np.uint32, 1, 36)[0])
    N = int(np.frombuffer(blob, np.uint32, 1, 20)[0])
    idx = np.frombuffer(blob, np.uint64, nb + 1, 128)
    rs = (128 + 8 * (nb + 1) + 15) & ~15
    for i in range(nb):
        h = np.frombuffer(blob, np.uint32, 3 + N, rs + int(idx[i]))
        yield int(h[1]), int(h[3])  # W, total symbols (cum of the finest child level)


def rule(n, k, wmax):
    if n == 0:
        return 0
    q = n // k
    return 1 if q < 1 else min(wmax, 1 << int(np.floor(np.log2(q))))


@pytest.mark.parametrize("k,wmax,b", [(64, 64, 5), (256, 64, 5), (1, 16, 5), (7, 32, 4), (64, 1, 5), (500, 64, 6)])
def test_each_record_width_follows_the_lane_rule(orc, k, wmax, b):
    # a uniform block (no symbols), two labels split by planes and a ball (few
    # symbols), dense Voronoi cells (many): widths from 0 to the maximum
    z, y, x = np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij")
    plane = np.where(x + 2 * y < 77, 1, 2).astype(np.uint32)
    ball = np.where((x - 20) ** 2 + (y - 33) ** 2 + (z - 9) ** 2 < 49, 5, 0).astype(np.uint32)
    vol = np.concatenate([np.zeros((64, 64, 64), np.uint32), plane, ball,
                          synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1)], axis=2)
    vol = np.ascontiguousarray(vol)
    blob = orc.encode_volume(vol, brick_log2=b, scale_bits=10, lane_k=k, lane_max=wmax)
    seen = set()
    for W, n in records(blob):
        assert W == rule(n, k, wmax), (W, n, k, wmax)
        seen.add(W)
    assert 0 in seen and len(seen) >= 2  # uniform bricks and coded ones
