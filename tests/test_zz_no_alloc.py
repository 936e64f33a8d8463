"""The decode entry point that allocates nothing (csv_decode_bricks_noalloc)
against csv_decode_bricks, through the C ABI: bit-identical output on two
calls in a row, the second with a smaller input, and the first large
enough to run in several chunks of the fixed scratch array."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import synth
from gpu_util import torch_cuda
from test_gpu_decode import golden_volume

pytestmark = pytest.mark.gpu


def log(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module")
def csvlib():
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    return csv


def _both(csv, pool, ids, lods=None, lod=0):
    """Output of csv_decode_bricks and of csv_decode_bricks_noalloc for the
    same requests, each into its own buffer pre-filled with -1."""
    import torch
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    if lods is None:
        tot = len(ids) * (32 >> lod) ** 3
        kw = {"lod": lod}
    else:
        lods = np.ascontiguousarray(lods, dtype=np.uint8)
        off, tot = csv.output_offsets(lods)
        kw = {"lods": torch.from_numpy(lods).cuda(), "out_offsets": torch.from_numpy(off.view(np.int64)).cuda()}
    want = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    got = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    pool.decode(d_ids, want, **kw)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    pool.decode_noalloc(d_ids, got, **kw)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    return got.cpu().numpy().view(np.uint32), want.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("shape", [None, (8, 3, 0, 1, 1)])
def test_noalloc_matches_decode_twice(csvlib, orc, shape):
    # one pool: the edge bricks (palettes beyond 252 and beyond the LDS
    # arena, so the global-arena kernel runs on the scratch's arenas; the
    # 32,768-label brick makes each request's slot about 47 KB, so 3000
    # requests take three chunks) and the 64^3 Voronoi volume
    edge = golden_volume()
    b_edge = orc.encode_volume(edge, scale_bits=11, lane_k=64)
    vor = synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1)
    b_vor = orc.encode_volume(vor, scale_bits=10, lane_k=64)
    pool = csvlib.Pool()
    assert pool.add_volume(b_edge) == 0
    assert pool.add_volume(b_vor) == 8
    if shape is not None:  # longest-first order: its bins live in the scratch too
        pool.set_shape(shape)
    rng = np.random.default_rng(77)
    n1 = 3000
    ids = rng.integers(0, 16, n1)
    lods = rng.integers(0, 6, n1)
    log("noalloc call 1: %d mixed-LOD requests" % n1)
    got, want = _both(csvlib, pool, ids, lods)
    np.testing.assert_array_equal(got, want)
    # the decode it is compared with agrees with the oracle on a sample
    pick = rng.choice(n1, 40, replace=False)
    off, _ = csvlib.output_offsets(np.asarray(lods, np.uint8))
    for i in pick:
        b, t = int(ids[i]), int(lods[i])
        ref = orc.decode_brick(b_edge, b, t) if b < 8 else orc.decode_brick(b_vor, b - 8, t)
        np.testing.assert_array_equal(got[off[i]:off[i] + ref.size], ref.ravel())
    # second call, smaller, one LOD for all (outputs packed back to back)
    ids2 = rng.integers(0, 16, 37)
    log("noalloc call 2: 37 requests at LOD 0")
    got2, want2 = _both(csvlib, pool, ids2, lod=0)
    np.testing.assert_array_equal(got2, want2)
    for k, b in enumerate(ids2[:8]):
        b = int(b)
        ref = orc.decode_brick(b_edge, b, 0) if b < 8 else orc.decode_brick(b_vor, b - 8, 0)
        np.testing.assert_array_equal(got2[k * 32768:(k + 1) * 32768], ref.ravel())


def test_noalloc_argument_errors(csvlib):
    import ctypes
    pool = csvlib.Pool()
    vor = synth.voronoi_bg(n=64, sites=50, bg=0.30, seed=2)
    pool.add_volume(csvlib.encode_volume(vor))
    L = csvlib.lib()
    vp = ctypes.c_void_p
    # n > 0 with no ids or output; a level of detail past 5; per-request
    # levels without offsets: rejected on the host before any launch
    assert L.csv_decode_bricks_noalloc(pool._p, None, None, 0, None, 4, None, None) == csvlib.CSV_EINVAL
    assert L.csv_decode_bricks_noalloc(pool._p, vp(16), None, 6, None, 1, vp(16), None) == csvlib.CSV_ERANGE
    assert L.csv_decode_bricks_noalloc(pool._p, vp(16), vp(16), 0, None, 1, vp(16), None) == csvlib.CSV_EINVAL
    assert L.csv_decode_bricks_noalloc(pool._p, None, None, 0, None, 0, None, None) == 0
