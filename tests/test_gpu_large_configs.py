"""GPU parity at the benchmark configurations' full sizes.

* 1024^3 neurite volume (32,768 bricks): every brick at full level of detail
  equals the source volume (the encoding is lossless, so the oracle's decode
  is the volume itself; a sample of bricks is also decoded by the oracle),
  and every brick at half level of detail equals the oracle's decode.
* 16,384 uneven requests over three volumes (the 64^3 Voronoi, the 512^3
  cells and the 512^3 blob volume), levels of detail drawn from {0, 1, 2},
  decoded in one persistent launch with the autotuned shape: every output
  equals the oracle's decode.
"""
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


def test_neurite_1024_full_and_half_lod(csvlib, orc):
    torch = torch_cuda()
    log("generating 1024^3 neurite volume")
    vol = synth.neurite(1024, 1024, 1024, labels=20000, seed=3)
    log("oracle encode")
    blob = orc.encode_volume(vol, scale_bits=10, lane_k=64)
    nb = 32 ** 3
    pool = csvlib.Pool()
    pool.add_volume(blob)
    ids = torch.arange(nb, dtype=torch.int32, device="cuda")
    # full LOD: the whole volume, compared on the device in brick order
    log("full LOD decode of %d bricks" % nb)
    out = torch.full((nb * 32768,), -1, dtype=torch.int32, device="cuda")
    pool.decode(ids, out, lod=0)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    ref = torch.from_numpy(vol.view(np.int32)).cuda()
    ref = ref.view(32, 32, 32, 32, 32, 32).permute(0, 2, 4, 1, 3, 5).reshape(-1)
    same = torch.equal(out, ref)
    if not same:
        bad = (out != ref).view(nb, -1).any(dim=1).nonzero().flatten()[:10].tolist()
        pytest.fail("full-LOD bricks differ from the volume, first: %s" % bad)
    del ref
    rng = np.random.default_rng(31)
    sample = np.sort(rng.choice(nb, 256, replace=False))
    got = out.view(nb, 32768)[torch.from_numpy(sample).cuda()].cpu().numpy().view(np.uint32).ravel()
    np.testing.assert_array_equal(got, orc.decode_bricks(blob, sample, np.zeros(256, np.uint8)))
    del out
    # half LOD: every brick against the oracle
    log("half LOD decode")
    half = torch.full((nb * 4096,), -1, dtype=torch.int32, device="cuda")
    pool.decode(ids, half, lod=1)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    want = orc.decode_bricks(blob, np.arange(nb), np.ones(nb, np.uint8))
    np.testing.assert_array_equal(half.cpu().numpy().view(np.uint32), want)


def record_sizes(blob):
    nb = int(np.frombuffer(blob, np.uint32, 1, 36)[0])
    idx = np.frombuffer(blob, np.uint64, nb + 1, 128)
    return np.diff(idx)


def test_mixed_16384_requests_autotuned(csvlib, orc):
    torch = torch_cuda()
    log("generating the three source volumes")
    vols = [synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1),
            synth.cells(n=512, grid=37, p_noise=0.5, seed=2),
            synth.blobs(n=512, sites=50, amp=24.0, seed=4)]
    blobs = [orc.encode_volume(v, scale_bits=10, lane_k=64) for v in vols]
    sizes = np.concatenate([record_sizes(b) for b in blobs])
    log("record sizes %d .. %d bytes" % (sizes.min(), sizes.max()))
    assert sizes.min() <= 64 and sizes.max() >= 4096
    pool = csvlib.Pool()
    first = [pool.add_volume(b) for b in blobs]
    counts = [len(record_sizes(b)) for b in blobs]
    rng = np.random.default_rng(5)
    n = 16384
    src = rng.integers(0, 3, n)
    local = np.array([rng.integers(0, counts[s]) for s in src], dtype=np.uint32)
    ids = (np.array(first, dtype=np.uint32)[src] + local).astype(np.uint32)
    lods = rng.integers(0, 3, n).astype(np.uint8)
    off, tot = csvlib.output_offsets(lods)
    want = np.empty(tot, np.uint32)
    for s in range(3):
        sel = np.nonzero(src == s)[0]
        dec = orc.decode_bricks(blobs[s], local[sel], lods[sel])
        pos = 0
        for i in sel:
            g = (32 >> int(lods[i])) ** 3
            want[off[i]:off[i] + g] = dec[pos:pos + g]
            pos += g
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_lods = torch.from_numpy(lods.copy()).cuda()
    d_off = torch.from_numpy(off.view(np.int64)).cuda()
    out = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    log("autotune over %d requests" % n)
    shape, ms = pool.autotune(d_ids, out, lods=d_lods, out_offsets=d_off, reps=3)
    log("tuned shape %s: %.3f ms" % (shape, ms))
    out.fill_(-1)
    pool.decode(d_ids, out, lods=d_lods, out_offsets=d_off)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), want)
