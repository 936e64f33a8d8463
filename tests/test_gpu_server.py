"""GPU tests of the serving loop: every completed brick equals the oracle's
decode of that brick alone, whatever else was in flight."""
import sys
import time

import numpy as np
import pytest

import synth
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def log(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module")
def setup(orc):
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    v1 = synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1)
    v2 = synth.cells(n=256, grid=19, seed=7)
    b1 = orc.encode_volume(v1, scale_bits=10, lane_k=64)
    b2 = orc.encode_volume(v2, scale_bits=10, lane_k=64)
    return csv, b1, b2


def wait_all(server, n, timeout=60.0):
    out, t0 = [], time.time()
    while sum(len(o) for o in out) < n:
        c = server.poll()
        if len(c):
            out.append(c.copy())
            yield c
        elif time.time() - t0 > timeout:
            raise TimeoutError("server completed %d of %d" % (sum(len(o) for o in out), n))
        else:
            time.sleep(0.0005)


def oracle_brick(orc, b1, b2, bid, lod):
    return (orc.decode_brick(b1, int(bid), int(lod)) if bid < 8 else orc.decode_brick(b2, int(bid) - 8, int(lod))).ravel()


@pytest.mark.parametrize("cache_mb,streams", [(256, 4), (2, 2)])
def test_alone_equals_mix(setup, orc, cache_mb, streams):
    csv, b1, b2 = setup
    pool = csv.Pool()
    pool.add_volume(b1)
    pool.add_volume(b2)
    n_b = 8 + 512
    rng = np.random.default_rng(cache_mb)
    n = 3000
    ids = rng.integers(0, n_b, n).astype(np.uint32)
    lods = rng.choice([0, 1, 2, 3, 5], n).astype(np.uint32)
    srv = csv.Server(pool, cache_bytes=cache_mb << 20, inflight_bytes=1 << 20, max_batch=256, streams=streams)
    log("server cache %d MiB, %d requests" % (cache_mb, n))
    seen = 0
    # submit in bursts so that requests arrive while others are on the GPU
    for k in range(0, n, 500):
        srv.submit(srv.requests(ids[k:k + 500], lods[k:k + 500], tags=np.arange(k, min(n, k + 500))))
    for comp in wait_all(srv, n):
        for c in comp:
            assert c["status"] == 0
            got = srv.read(c)
            np.testing.assert_array_equal(got, oracle_brick(orc, b1, b2, c["brick_id"], c["lod"]))
            assert c["brick_id"] == ids[c["tag"]] and c["lod"] == lods[c["tag"]]
            seen += 1
    assert seen == n
    st = srv.stats()
    log("stats %s" % {k: st[k] for k in ("hits", "misses", "joined", "evictions", "rebuilds", "p50_us", "p99_us")})
    assert st["completed"] == n and st["hits"] + st["misses"] + st["joined"] == n
    if cache_mb == 2:
        assert st["evictions"] + st["rebuilds"] > 0
    srv.close()


def test_bad_requests(setup):
    csv, b1, b2 = setup
    pool = csv.Pool()
    pool.add_volume(b1)
    srv = csv.Server(pool, cache_bytes=16 << 20)
    srv.submit(srv.requests([3, 99, 2], [0, 0, 6], tags=[0, 1, 2]))
    got = {}
    for comp in wait_all(srv, 3):
        for c in comp:
            got[int(c["tag"])] = int(c["status"])
    assert got == {0: 0, 1: csv.CSV_ERANGE, 2: csv.CSV_ERANGE}
    srv.close()


def test_visibility_table_skips_invisible_bricks(setup, orc):
    # the visibility of every brick comes from csv_bricks_visible under a
    # transfer function showing a few labels; requests for the invisible
    # bricks complete as skipped, the others decode to the oracle's bytes,
    # and clearing the table decodes everything again
    csv, b1, b2 = setup
    torch = torch_cuda()
    pool = csv.Pool()
    pool.add_volume(b1)
    pool.add_volume(b2)
    n_b = 8 + 512
    n_lab = 19 ** 3 + 1
    show = np.zeros(n_lab, bool)
    show[np.random.default_rng(3).choice(n_lab, 60, replace=False)] = True
    words = np.zeros((n_lab + 31) // 32, np.uint32)
    for lab in np.nonzero(show)[0]:
        words[lab >> 5] |= np.uint32(1 << (lab & 31))
    d_ids = torch.arange(n_b, dtype=torch.int32, device="cuda")
    vis = pool.visible(d_ids, torch.from_numpy(words.view(np.int32)).cuda(), n_lab).cpu().numpy()
    assert 0 < vis.sum() < n_b
    srv = csv.Server(pool, cache_bytes=64 << 20, max_batch=128)
    srv.set_visible(vis)
    rng = np.random.default_rng(9)
    ids = rng.integers(0, n_b, 1500).astype(np.uint32)
    lods = rng.choice([0, 1, 3], 1500).astype(np.uint32)
    srv.submit(srv.requests(ids, lods, tags=np.arange(1500)))
    skipped = 0
    for comp in wait_all(srv, 1500):
        for c in comp:
            assert c["status"] == 0 and c["brick_id"] == ids[c["tag"]]
            if vis[c["brick_id"]]:
                assert c["skipped"] == 0
                np.testing.assert_array_equal(srv.read(c), oracle_brick(orc, b1, b2, c["brick_id"], c["lod"]))
            else:
                assert c["skipped"] == 1 and c["data"] == 0 and c["elems"] == 0
                skipped += 1
    assert skipped == int((vis[ids] == 0).sum()) and srv.stats()["skipped"] == skipped
    srv.set_visible(None)
    hidden = np.nonzero(vis == 0)[0][:50].astype(np.uint32)
    srv.submit(srv.requests(hidden, np.zeros(len(hidden), np.uint32)))
    for comp in wait_all(srv, len(hidden)):
        for c in comp:
            assert c["skipped"] == 0
            np.testing.assert_array_equal(srv.read(c), oracle_brick(orc, b1, b2, c["brick_id"], 0))
    with pytest.raises(Exception):
        srv.set_visible(np.ones(n_b + 1, np.uint8))
    srv.close()


def test_trace_replay(setup, orc):
    csv, b1, b2 = setup
    pool = csv.Pool()
    pool.add_volume(b2)
    rng = np.random.default_rng(3)
    n = 20000
    reqs = csv.Server.requests(rng.integers(0, 512, n), rng.integers(0, 3, n),
                               t_arrival_ns=np.sort(rng.uniform(0, 0.05e9, n)).astype(np.uint64))
    srv = csv.Server(pool, cache_bytes=512 << 20, max_batch=1024, streams=4)
    log("trace replay %d requests" % n)
    done, got = srv.run_trace(reqs, collect=True, timeout_s=20)
    assert got == n and (done["status"] == 0).all()
    st = srv.stats()
    log("trace p50 %.1f us p99 %.1f us" % (st["p50_us"], st["p99_us"]))
    srv.close()


def test_big_palette_bricks_on_four_streams(orc):
    # most bricks have palettes above 252 entries and take the leaf kernel's
    # global-memory arenas; small batches on 4 streams overlap on the GPU
    # (each stream has arenas of its own), and a 6 MiB cache evicts and
    # decodes again.  Every completion equals the oracle's decode.
    torch_cuda()
    import paper_2308_16619_amd as csv
    rng = np.random.default_rng(21)
    noisy = rng.integers(1, 4000, size=(64, 64, 192)).astype(np.uint32)  # P about 3000
    vol = np.ascontiguousarray(np.concatenate([noisy, synth.voronoi_bg(n=64, sites=60, seed=2)], axis=2))
    blob = orc.encode_volume(vol, scale_bits=10, lane_k=64)
    pool = csv.Pool()
    pool.add_volume(blob)
    nb = 4 * 8
    n = 1200
    ids = rng.integers(0, nb, n).astype(np.uint32)
    lods = rng.choice([0, 0, 0, 1, 2], n).astype(np.uint32)
    srv = csv.Server(pool, cache_bytes=6 << 20, inflight_bytes=1 << 20, max_batch=2, streams=4)
    log("big palettes, 4 streams, %d requests" % n)
    for k in range(0, n, 100):
        srv.submit(srv.requests(ids[k:k + 100], lods[k:k + 100], tags=np.arange(k, min(n, k + 100))))
    seen = 0
    want = {}
    for comp in wait_all(srv, n, timeout=120):
        for c in comp:
            assert c["status"] == 0
            key = (int(c["brick_id"]), int(c["lod"]))
            if key not in want:
                want[key] = orc.decode_brick(blob, key[0], key[1]).ravel()
            np.testing.assert_array_equal(srv.read(c), want[key])
            seen += 1
    st = srv.stats()
    log("stats %s" % {k: st[k] for k in ("misses", "batches", "evictions", "rebuilds")})
    assert seen == n and st["batches"] > 20 and st["failed"] == 0
    srv.close()


def test_failed_decode_is_reported_and_not_cached(setup, orc):
    # a record with a flipped word-stream bit fails on the device: its
    # requests complete with CSV_ECORRUPT every time (nothing is cached),
    # the other bricks of the same batches decode to the oracle's bytes
    csv, b1, b2 = setup
    B = 8
    idx = np.frombuffer(b1, np.uint64, B + 1, 128)
    rs = (128 + 8 * (B + 1) + 15) & ~15
    w = np.frombuffer(b1, np.uint32, 8, rs + int(idx[4]))
    bad = bytearray(b1)
    bad[rs + int(idx[4]) + 4 * (8 + int(w[0]) + int(w[1])) + 2 * (int(w[2]) // 2)] ^= 0x10
    pool = csv.Pool()
    pool.add_volume(bytes(bad))
    srv = csv.Server(pool, cache_bytes=64 << 20, max_batch=8)
    for rnd in range(2):
        ids = np.array([3, 4, 5, 4, 0], np.uint32)
        srv.submit(srv.requests(ids, np.zeros(5, np.uint32), tags=np.arange(5)))
        for comp in wait_all(srv, 5):
            for c in comp:
                if c["brick_id"] == 4:
                    assert c["status"] == csv.CSV_ECORRUPT and c["data"] == 0 and c["hit"] == 0
                else:
                    assert c["status"] == 0
                    np.testing.assert_array_equal(srv.read(c), orc.decode_brick(b1, int(c["brick_id"]), 0).ravel())
    st = srv.stats()
    assert st["failed"] >= 2 and st["error"] == csv.CSV_ECORRUPT
    srv.close()
