"""GPU: detail separation (Sec. 4.2).  A volume added with CSV_DETAIL_HOST
keeps in HBM each record only up to the words its level-1 prefix reads
(the prefix property of the stream, Sec. 3.4); level-0 detail lives in
pinned host memory and is staged on demand.

Expectations come from the oracle alone: decodes at every LOD, and which
bricks split and how many detail bytes go to the host, from the oracle's own
rANS decoder (words consumed by the first c_1 symbols of each record)."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import gpu_decode, torch_cuda

pytestmark = pytest.mark.gpu

HDR = 8  # u32 words before the palette: P, W, n_words, c_0 .. c_4


def log(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def csvlib():
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    return csv


@pytest.fixture(scope="module")
def volumes(orc):
    # config 1 (64^3, background plus 200 labels), the edge bricks (uniform,
    # checkerboard, P > 32768 for the global-arena path, ...), and a 128^3
    # cut of the cells volume
    from test_gpu_decode import golden_volume
    vols = [synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1), golden_volume(),
            synth.cells(n=512, grid=37, seed=2)[:128, :128, :128].copy()]
    return [orc.encode_volume(v, scale_bits=10, lane_k=64) for v in vols]


def split_plan(orc, blob):
    """Per brick: the detail bytes that go to host memory (0: whole record kept)."""
    info = orc.volume_info(blob)
    nb = info["n_bricks"]
    index = np.frombuffer(blob, dtype=np.uint64, count=nb + 1, offset=128)
    rs = (128 + 8 * (nb + 1) + 15) & ~15
    det = np.zeros(nb, np.int64)
    for i in range(nb):
        rec = np.frombuffer(blob, dtype=np.uint32, count=HDR, offset=rs + int(index[i]))
        P, W, nw, c0, c1 = (int(v) for v in rec[:5])
        if c0 == 0:
            continue
        st = np.frombuffer(blob, dtype=np.uint32, count=W, offset=rs + int(index[i]) + 4 * (HDR + P))
        words = np.frombuffer(blob, dtype=np.uint16, count=nw, offset=rs + int(index[i]) + 4 * (HDR + P + W))
        sym, _, used = orc.rans_decode(st, words, c1, info["freq"], info["scale_bits"], tab_split=c1)
        ndw, pfx = (nw + 1) // 2, (used + 1) // 2
        if pfx < ndw:
            det[i] = 4 * (ndw - pfx)
    return det


def up2(block):
    return block.repeat(2, 0).repeat(2, 1).repeat(2, 2)


def fallback(orc, blob, ids, det):
    """Full-LOD output when no detail is staged: level 0 for whole records,
    level 1 upsampled 2x for split ones."""
    out = []
    for i in ids:
        if det[i]:
            out.append(up2(orc.decode_brick(blob, int(i), 1)).reshape(-1))
        else:
            out.append(orc.decode_brick(blob, int(i), 0).reshape(-1))
    return np.concatenate(out)


def split_pool(csvlib, blobs, detail=(True, True, True)):
    pool = csvlib.Pool()
    firsts = [pool.add_volume(b, detail_host=d) for b, d in zip(blobs, detail)]
    assert pool.last_error() == (0, 0)
    return pool, firsts


def test_split_bytes_and_coarse_lods(csvlib, orc, volumes):
    plans = [split_plan(orc, b) for b in volumes]
    assert all(p.sum() > 0 for p in (plans[0], plans[2]))
    whole = csvlib.Pool()
    for b in volumes:
        whole.add_volume(b)
    pool, firsts = split_pool(csvlib, volumes)
    wi, si = whole.info(), pool.info()
    log("device bytes %d -> %d, host bytes %d" % (wi["device_bytes"], si["device_bytes"], si["host_bytes"]))
    assert wi["host_bytes"] == 0
    assert si["host_bytes"] == sum(int(p.sum()) for p in plans)
    # levels >= 1 decode exactly from the device prefix
    for f, b in zip(firsts, volumes):
        nb = orc.volume_info(b)["n_bricks"]
        for t in range(1, 6):
            log("split pool, volume at %d, lod %d" % (f, t))
            got, _ = gpu_decode(pool, f + np.arange(nb), t)
            np.testing.assert_array_equal(got, orc.decode_bricks(b, np.arange(nb), [t] * nb))
    rng = np.random.default_rng(5)
    ids = rng.integers(0, firsts[2], 400)  # volumes 0 and 1 only (their bricks: ids 0 .. 15)
    lods = rng.integers(1, 6, 400)
    got, _ = gpu_decode(pool, ids, lods)
    want = np.concatenate([orc.decode_bricks(volumes[0] if i < 8 else volumes[1], [i % 8], [t])
                           for i, t in zip(ids, lods)])
    np.testing.assert_array_equal(got, want)


def test_full_lod_without_detail_falls_back(csvlib, orc, volumes):
    pool, firsts = split_pool(csvlib, volumes)
    for f, b in zip(firsts, volumes):
        det = split_plan(orc, b)
        nb = len(det)
        log("unstaged full LOD, volume at %d (%d of %d bricks split)" % (f, int((det > 0).sum()), nb))
        got, err = gpu_decode(pool, f + np.arange(nb), 0, check_error=False)
        np.testing.assert_array_equal(got, fallback(orc, b, np.arange(nb), det))
        if det.any():
            assert err[0] == csvlib.CSV_EDETAIL and det[err[1] - f] > 0, err
        else:
            assert err == (0, 0)


def test_staged_detail_decodes_exactly(csvlib, orc, volumes):
    torch = torch_cuda()
    pool, firsts = split_pool(csvlib, volumes)
    pool.set_detail_staging(64 << 20)
    n = pool.info()["n_bricks"]
    stream = torch.cuda.current_stream()
    done = pool.stage_detail(np.arange(n), stream)
    assert done == n
    for f, b in zip(firsts, volumes):
        nb = orc.volume_info(b)["n_bricks"]
        log("staged full LOD, volume at %d" % f)
        got, _ = gpu_decode(pool, f + np.arange(nb), 0)
        np.testing.assert_array_equal(got, orc.decode_bricks(b, np.arange(nb), [0] * nb))
        rng = np.random.default_rng(f + 11)
        ids = rng.integers(0, nb, 300)
        lods = rng.integers(0, 6, 300)
        got, _ = gpu_decode(pool, f + ids, lods)
        np.testing.assert_array_equal(got, orc.decode_bricks(b, ids, lods))
        # the one-launch-per-brick path reads the same staged detail
        got, _ = gpu_decode(pool, f + ids[:12], lods[:12], plain=True)
        np.testing.assert_array_equal(got, orc.decode_bricks(b, ids[:12], lods[:12]))
    # staging twice is a no-op; a resize needs the staged detail released
    assert pool.stage_detail(np.arange(n), stream) == n
    with pytest.raises(RuntimeError):
        pool.set_detail_staging(32 << 20)
    pool.release_detail(stream)
    b, f = volumes[2], firsts[2]
    det = split_plan(orc, b)
    got, err = gpu_decode(pool, f + np.arange(len(det)), 0, check_error=False)
    np.testing.assert_array_equal(got, fallback(orc, b, np.arange(len(det)), det))
    assert err[0] == csvlib.CSV_EDETAIL


def test_staging_capacity_and_order(csvlib, orc, volumes):
    torch = torch_cuda()
    b = volumes[2]
    det = split_plan(orc, b)
    nb = len(det)
    pool = csvlib.Pool()
    pool.add_volume(volumes[1])  # ordinary volume first: its bricks need no staging
    f = pool.add_volume(b, detail_host=True)
    cap = 4096 * 8
    pool.set_detail_staging(cap)
    stream = torch.cuda.current_stream()
    order = np.random.default_rng(9).permutation(nb)
    # expected: bricks taken in order while their 16-byte aligned detail fits
    used, want_done = 0, nb
    for k, i in enumerate(order):
        need = (int(det[i]) + 15) & ~15
        if used + need > cap:
            want_done = k
            break
        used += need
    done = pool.stage_detail(np.concatenate([[0, 3], f + order]), stream)
    log("staging %d bytes: %d of %d bricks" % (cap, done - 2, nb))
    assert done - 2 == want_done and want_done < nb
    got, err = gpu_decode(pool, f + order, 0, check_error=False)
    head = order[:want_done]
    expect = np.concatenate([orc.decode_bricks(b, head, [0] * len(head)),
                             fallback(orc, b, order[want_done:], det)])
    np.testing.assert_array_equal(got, expect)
    assert err[0] == (csvlib.CSV_EDETAIL if det[order[want_done:]].any() else 0)
    # a bad id stops staging at its index
    pool.release_detail(stream)
    with pytest.raises(RuntimeError):
        pool.stage_detail([f, f + 1, 10 ** 6], stream)
    got, _ = gpu_decode(pool, [0, 1], 0)
    np.testing.assert_array_equal(got, orc.decode_bricks(volumes[1], [0, 1], [0, 0]))
    # the ordinary volume still decodes whole after the split volume was added
    got, _ = gpu_decode(pool, np.arange(8), 0)
    np.testing.assert_array_equal(got, orc.decode_bricks(volumes[1], np.arange(8), [0] * 8))


def test_split_then_ordinary_volume(csvlib, orc, volumes):
    # a volume added after a split one keeps whole records; both decode
    pool, firsts = split_pool(csvlib, volumes, detail=(True, False, True))
    rng = np.random.default_rng(21)
    for f, b, split in zip(firsts, volumes, (True, False, True)):
        nb = orc.volume_info(b)["n_bricks"]
        ids = rng.integers(0, nb, 200)
        lods = rng.integers(1 if split else 0, 6, 200)
        log("mixed pool, volume at %d" % f)
        got, _ = gpu_decode(pool, f + ids, lods)
        np.testing.assert_array_equal(got, orc.decode_bricks(b, ids, lods))


def wait_all(server, n, timeout=60.0):
    import time
    got, t0 = 0, time.time()
    while got < n:
        c = server.poll()
        if len(c):
            got += len(c)
            yield c
        elif time.time() - t0 > timeout:
            raise TimeoutError("server completed %d of %d" % (got, n))
        else:
            time.sleep(0.0005)


@pytest.mark.parametrize("staging", [8 << 20, 16 << 10, 4096])
def test_server_stages_detail(csvlib, orc, volumes, staging):
    # the serving loop over a pool with level-0 detail in host memory: every
    # full-LOD brick is decoded exactly (its detail staged for its batch),
    # except bricks whose detail exceeds the staging buffer (CSV_EDETAIL)
    pool = csvlib.Pool()
    f_plain = pool.add_volume(volumes[0])
    f_cells = pool.add_volume(volumes[2], detail_host=True)
    f_edge = pool.add_volume(volumes[1], detail_host=True)
    blobs = {f_plain: volumes[0], f_cells: volumes[2], f_edge: volumes[1]}
    det = np.concatenate([np.zeros(8, np.int64), split_plan(orc, volumes[2]), split_plan(orc, volumes[1])])
    det16 = (det + 15) & ~15
    assert pool.info()["host_bytes"] == int(det.sum())
    pool.set_detail_staging(staging)
    n_b = len(det)
    rng = np.random.default_rng(staging % 1000 + 3)
    n = 2500
    ids = rng.integers(0, n_b, n).astype(np.uint32)
    lods = rng.choice([0, 0, 0, 1, 2, 5], n).astype(np.uint32)
    srv = csvlib.Server(pool, cache_bytes=64 << 20, inflight_bytes=1 << 20, max_batch=64, streams=3)
    log("serving a split pool, staging %d bytes, %d requests" % (staging, n))
    for k in range(0, n, 500):
        srv.submit(srv.requests(ids[k:k + 500], lods[k:k + 500], tags=np.arange(k, min(n, k + 500))))
    seen = edetail = 0
    for comp in wait_all(srv, n):
        for c in comp:
            b, t = int(c["brick_id"]), int(c["lod"])
            first = max(f for f in blobs if f <= b)
            if t == 0 and det16[b] > staging:
                assert c["status"] == csvlib.CSV_EDETAIL, (b, c["status"])
                edetail += 1
            else:
                assert c["status"] == 0, (b, t, c["status"])
                np.testing.assert_array_equal(srv.read(c), orc.decode_brick(blobs[first], b - first, t).ravel())
            seen += 1
    st = srv.stats()
    srv.close()
    log("stats %s" % {k: st[k] for k in ("hits", "misses", "stall_staging", "detail_staged_bytes",
                                         "detail_releases", "p99_us")})
    assert seen == n and st["error"] == 0
    assert st["detail_staged_bytes"] > 0 and st["detail_releases"] > 0
    assert (edetail > 0) == bool((det16[ids[lods == 0]] > staging).any())
    assert pool.last_error() == (0, 0)
