"""GPU parity of the serving pool at full size: the 2048x2048x1024 neurite
volume (131,072 bricks) resident in HBM, with a 16 GiB decoded-brick LRU
cache and a 16 GiB frame cache filled by every brick at full LOD, so that
cache offsets run past 2^31 labels (8 GiB).  A sample of cached bricks,
most of them past that mark, is read back and compared with the oracle's
decode of the brick alone."""
import sys
import time

import numpy as np
import pytest

import synth
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

NX, NY, NZ = 2048, 2048, 1024
NB = (NX // 32) * (NY // 32) * (NZ // 32)
GIB16 = 16 << 30


def log(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big(orc):
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    log("generating the %dx%dx%d neurite volume" % (NX, NY, NZ))
    vol = synth.neurite(NX, NY, NZ, labels=80000, seed=8)
    log("oracle encode")
    blob = orc.encode_volume(vol, scale_bits=10, lane_k=64)
    del vol
    pool = csv.Pool()
    pool.add_volume(blob)
    return csv, blob, pool


def sample(rng, offsets_elems, k_high=1500, k_low=500):
    """Indices of k_high entries at element offsets >= 2^31 and k_low below."""
    hi = np.nonzero(offsets_elems >= (1 << 31))[0]
    lo = np.nonzero(offsets_elems < (1 << 31))[0]
    assert len(hi) >= k_high
    return np.concatenate([rng.choice(hi, k_high, replace=False), rng.choice(lo, k_low, replace=False)])


def test_server_16gib_cache_every_brick(big, orc):
    csv, blob, pool = big
    srv = csv.Server(pool, cache_bytes=GIB16, inflight_bytes=1 << 30, max_batch=4096, streams=4)
    base = srv.cache_ptr()
    ids = np.arange(NB, dtype=np.uint32)
    rng = np.random.default_rng(41)
    srv.submit(srv.requests(ids, np.zeros(NB, np.uint32), tags=ids))
    log("serving all %d bricks at full LOD into a 16 GiB cache" % NB)
    # completions are valid until the next poll: the sampled ones are read at once
    got = {}
    n_done, t0 = 0, time.time()
    seen_off = np.zeros(NB, np.int64)
    picked = set(rng.choice(NB, 4000, replace=False).tolist())
    while n_done < NB:
        comp = srv.poll()
        if not len(comp):
            assert time.time() - t0 < 300, "server completed %d of %d" % (n_done, NB)
            time.sleep(0.001)
            continue
        assert (comp["status"] == 0).all()
        for c in comp:
            off = (int(c["data"]) - base) // 4
            seen_off[int(c["tag"])] = off
            if int(c["tag"]) in picked or (off >= (1 << 31) and len(got) < 3000 and rng.random() < 0.05):
                got[int(c["tag"])] = (off, srv.read(c))
        n_done += len(comp)
    st = srv.stats()
    log("done: %d misses, cache used %.2f GiB" % (st["misses"], st["cache_bytes_used"] / 2 ** 30))
    assert st["misses"] == NB and st["failed"] == 0
    assert seen_off.max() + 32768 <= GIB16 // 4
    keys = np.array(sorted(got))
    offs = np.array([got[k][0] for k in keys])
    chosen = keys[sample(rng, offs)]
    log("comparing %d bricks (max offset %d elements)" % (len(chosen), offs.max()))
    want = orc.decode_bricks(blob, chosen.astype(np.uint32), np.zeros(len(chosen), np.uint8)).reshape(-1, 32768)
    for i, k in enumerate(chosen):
        np.testing.assert_array_equal(got[int(k)][1], want[i], err_msg="brick %d at %d" % (k, got[int(k)][0]))
    srv.close()


def test_frame_cache_16gib_every_brick(big, orc):
    csv, blob, pool = big
    torch = torch_cuda()
    fc = csv.FrameCache(pool, GIB16, NB)
    ids = torch.arange(NB, dtype=torch.int32, device="cuda")
    lods = torch.zeros(NB, dtype=torch.uint8, device="cuda")
    log("one frame of all %d bricks at full LOD into a 16 GiB frame cache" % NB)
    slots, st = fc.frame(ids, lods)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    assert st["decoded"] == NB and st["rebuilt"] in (0, 1)
    s = slots.cpu().numpy()
    assert (s >= 0).all() and s.max() + 32768 <= GIB16 // 4
    rng = np.random.default_rng(43)
    chosen = sample(rng, s)
    log("comparing %d bricks (max offset %d elements)" % (len(chosen), s[chosen].max()))
    want = orc.decode_bricks(blob, chosen.astype(np.uint32), np.zeros(len(chosen), np.uint8)).reshape(-1, 32768)
    for i, r in enumerate(chosen):
        np.testing.assert_array_equal(fc.read(int(s[r]), 32768), want[i], err_msg="brick %d at %d" % (r, s[r]))
    fc.close()
