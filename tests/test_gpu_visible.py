"""GPU: the empty-space test of requested bricks (Sec. 4, empty-space
skipping) against its definition: a brick is visible when one of its labels
has its bit set in the visibility bitset (labels beyond the bitset are
invisible).  The expected masks come from the source volumes themselves
(each brick's distinct labels), not from the codec."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def log(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def csvlib():
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    return csv


def brick_labels(vol):
    """Distinct labels of every 32^3 brick, in pool order (x fastest)."""
    nz, ny, nx = vol.shape
    out = []
    for bz in range(nz // 32):
        for by in range(ny // 32):
            for bx in range(nx // 32):
                b = vol[32 * bz:32 * (bz + 1), 32 * by:32 * (by + 1), 32 * bx:32 * (bx + 1)]
                out.append(np.unique(b))
    return out


def pack_bits(vis):
    """bool[n] -> uint32 words, bit (label & 31) of word label >> 5."""
    w = np.zeros(max((len(vis) + 31) // 32, 1), np.uint32)
    idx = np.nonzero(vis)[0].astype(np.uint64)
    np.bitwise_or.at(w, (idx >> 5).astype(np.int64), (np.uint64(1) << (idx & np.uint64(31))).astype(np.uint32))
    return w


def expected(labels, ids, vis):
    n = len(vis)
    return np.array([1 if (lab[lab < n].size and vis[lab[lab < n]].any()) else 0
                     for lab in (labels[i] for i in ids)], np.uint8)


def run(torch, pool, ids, vis):
    d_ids = torch.from_numpy(np.asarray(ids, np.uint32).view(np.int32)).cuda()
    n_bits = len(vis)
    bits = torch.from_numpy(pack_bits(vis).view(np.int32)).cuda() if n_bits else None
    got = pool.visible(d_ids, bits, n_bits)
    torch.cuda.synchronize()
    return got.cpu().numpy()


@pytest.fixture(scope="module")
def volumes(orc):
    # config 1 (background 0 plus 200 labels), the edge bricks (uniform,
    # two labels, checkerboard, >32k distinct labels, zero), and a 256^3 cut
    # of the cells volume
    from test_gpu_decode import golden_volume
    vols = [synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1), golden_volume(),
            synth.cells(n=512, grid=37, seed=2)[:256, :256, :256].copy()]
    blobs = [orc.encode_volume(v, scale_bits=10, lane_k=64) for v in vols]
    return vols, blobs


@pytest.mark.parametrize("density", [0.0, 0.002, 0.05, 0.5, 1.0])
def test_visibility_matches_definition(csvlib, volumes, density):
    torch = torch_cuda()
    vols, blobs = volumes
    pool = csvlib.Pool()
    first = [pool.add_volume(b) for b in blobs]
    labels = []
    for v in vols:
        labels += brick_labels(v)
    n_labels = int(max(v.max() for v in vols)) + 1
    rng = np.random.default_rng(int(density * 1000) + 7)
    ids = np.concatenate([np.arange(len(labels)), rng.integers(0, len(labels), 3000)]).astype(np.uint32)
    for n_bits in (n_labels, n_labels // 3, 0):
        vis = rng.random(n_bits) < density
        log("visibility density %g, %d label bits, %d requests" % (density, n_bits, len(ids)))
        got = run(torch, pool, ids, vis)
        np.testing.assert_array_equal(got, expected(labels, ids, vis))
        assert pool.last_error() == (0, 0)
    assert first[0] == 0


def test_background_only_and_errors(csvlib, volumes):
    torch = torch_cuda()
    vols, blobs = volumes
    pool = csvlib.Pool()
    pool.add_volume(blobs[0])
    labels = brick_labels(vols[0])
    # only label 0 visible: exactly the bricks that contain background
    vis = np.zeros(256, bool)
    vis[0] = True
    got = run(torch, pool, np.arange(8), vis)
    np.testing.assert_array_equal(got, [1 if 0 in lab else 0 for lab in labels])
    # an unknown brick id gives 0 and a range error naming the request
    got = run(torch, pool, [3, 8, 5], np.ones(256, bool))
    np.testing.assert_array_equal(got, [1, 0, 1])
    assert pool.last_error() == (csvlib.CSV_ERANGE, 1)
    # no requests: nothing to do
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    assert pool.visible(empty, None, 0).numel() == 0
