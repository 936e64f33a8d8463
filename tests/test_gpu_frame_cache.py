"""GPU: the frame cache (Sec. 4.1).  Every stored block equals the oracle's
decode of its brick; the per-frame counts equal a host model of the
allocator (free blocks per LOD, top pointer, rebuild when the top would
pass the end); blocks of one frame never overlap; invisible and LOD-5
requests are not stored.  Visibility comes from the volumes' own labels."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def log(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


def block_elems(t):
    return 1 << (3 * (4 - t))


@pytest.fixture(scope="module")
def setup(orc):
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    vols = [synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1),
            synth.cells(n=512, grid=37, seed=2)[:256, :256, :256].copy()]
    blobs = [orc.encode_volume(v, scale_bits=10, lane_k=64) for v in vols]
    labels = []
    for v in vols:
        nz, ny, nx = v.shape
        for bz in range(nz // 32):
            for by in range(ny // 32):
                for bx in range(nx // 32):
                    labels.append(np.unique(v[32 * bz:32 * bz + 32, 32 * by:32 * by + 32, 32 * bx:32 * bx + 32]))
    return csv, blobs, labels


class Model:
    """Host model of the cache's bookkeeping (counts only)."""

    def __init__(self, cap_elems):
        self.cap = cap_elems
        self.cached = set()
        self.free = [0] * 5
        self.top = 0

    def frame(self, keys):
        evicted = self.cached - keys
        for (_, t) in evicted:
            self.free[t] += 1
        new = keys - self.cached
        need = sum(max(0, sum(1 for k in new if k[1] == t) - self.free[t]) * block_elems(t) for t in range(5))
        rebuilt = self.top + need > self.cap
        if rebuilt:
            self.free = [0] * 5
            self.top = sum(block_elems(t) for (_, t) in keys)
            decoded = len(keys)
            error = self.top > self.cap
            if error:
                self.top = 0
                self.cached = set()
                return dict(decoded=0, evicted=len(evicted), rebuilt=1, error=True, used=0)
        else:
            for t in range(5):
                m = sum(1 for k in new if k[1] == t)
                take = min(m, self.free[t])
                self.free[t] -= take
                self.top += (m - take) * block_elems(t)
            decoded = len(new)
        self.cached = set(keys)
        return dict(decoded=decoded, evicted=len(evicted), rebuilt=int(rebuilt), error=False, used=self.top)


def decode_ref(orc, blobs, bid, t):
    return (orc.decode_brick(blobs[0], bid, t) if bid < 8 else orc.decode_brick(blobs[1], bid - 8, t)).ravel()


def frames(n_bricks, n_frames, seed):
    """Requests of a moving window over the brick ids (consecutive frames
    overlap), with repeats, LODs weighted toward coarse levels, and a few
    unknown ids."""
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n_frames):
        lo = (f * n_bricks // (2 * n_frames)) % n_bricks
        ids = (lo + rng.integers(0, n_bricks // 3, 400)) % n_bricks
        lods = rng.choice(6, 400, p=[0.1, 0.2, 0.25, 0.2, 0.15, 0.1])
        ids[rng.integers(0, 400, 3)] = n_bricks + 5
        out.append((ids.astype(np.uint32), lods.astype(np.uint8)))
    return out


def run_frames(csv, orc, blobs, labels, cap_bytes, n_frames=8, seed=3, density=None, expect_error=False, sync=True):
    """sync False: frames without statistics (no wait for the device), the
    statistics read afterwards with last_stats()."""
    torch = torch_cuda()
    pool = csv.Pool()
    for b in blobs:
        pool.add_volume(b)
    nb = len(labels)
    cache = csv.FrameCache(pool, cap_bytes, 512)
    model = Model(cap_bytes // 32)
    n_lab = int(max(l.max() for l in labels)) + 1
    stats_all = []
    for f, (ids, lods) in enumerate(frames(nb, n_frames, seed)):
        d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
        d_lods = torch.from_numpy(lods).cuda()
        vis = np.ones(len(ids), bool)
        bits = None
        if density is not None and f % 2 == 1:
            show = np.random.default_rng(100 + f).random(n_lab) < density
            words = np.zeros((n_lab + 31) // 32, np.uint32)
            idx = np.nonzero(show)[0].astype(np.uint64)
            np.bitwise_or.at(words, (idx >> 5).astype(np.int64), (np.uint64(1) << (idx & np.uint64(31))).astype(np.uint32))
            bits = torch.from_numpy(words.view(np.int32)).cuda()
            vis = np.array([i < nb and bool(show[labels[i]].any()) for i in ids])
        keys = {(int(i), int(t)) for i, t, v in zip(ids, lods, vis) if i < nb and t < 5 and v}
        want = model.frame(keys)
        log("frame %d: %d requests, %d distinct keys, cache %d bytes" % (f + 1, len(ids), len(keys), cap_bytes))
        if want["error"]:
            if sync:
                with pytest.raises(csv.CsvError) as e:
                    cache.frame(d_ids, d_lods, bits, n_lab if bits is not None else 0)
            else:
                slots, st = cache.frame(d_ids, d_lods, bits, n_lab if bits is not None else 0, stats=False)
                assert st is None
                with pytest.raises(csv.CsvError) as e:
                    cache.last_stats()
                assert (slots.cpu().numpy() == -1).all()
            assert e.value.code == csv.CSV_ENOMEM
            assert expect_error
            pool.last_error()
            continue
        slots, st = cache.frame(d_ids, d_lods, bits, n_lab if bits is not None else 0, stats=sync)
        if not sync:
            assert st is None
            st = cache.last_stats()
        torch.cuda.synchronize()
        pool.last_error()  # unknown ids are reported by the visibility test; the cache skips them
        assert st["frame"] == f + 1 and st["requests"] == len(ids)
        assert st["distinct"] == len(keys)
        assert (st["decoded"], st["evicted"], st["rebuilt"]) == (want["decoded"], want["evicted"], want["rebuilt"]), (st, want)
        assert st["hits"] == len(keys) - want["decoded"]
        assert st["used_bytes"] == want["used"] * 32
        slots = slots.cpu().numpy()
        seen = {}
        for i, t, v, s in zip(ids.tolist(), lods.tolist(), vis.tolist(), slots.tolist()):
            stored = i < nb and t < 5 and v
            assert (s >= 0) == stored, (i, t, v, s)
            if not stored:
                continue
            k = (int(i), int(t))
            if k in seen:
                assert seen[k] == s
                continue
            seen[k] = int(s)
            n = (32 >> t) ** 3
            assert s % 8 == 0 and s + n <= cap_bytes // 4
            np.testing.assert_array_equal(cache.read(s, n), decode_ref(orc, blobs, int(i), int(t)))
        iv = sorted((s, s + (32 >> t) ** 3) for (i, t), s in seen.items())
        assert all(a[1] <= b[0] for a, b in zip(iv, iv[1:])), "blocks overlap"
        stats_all.append(st)
    cache.close()
    return stats_all


def test_frames_large_cache(setup, orc):
    csv, blobs, labels = setup
    st = run_frames(csv, orc, blobs, labels, 256 << 20)
    assert sum(s["hits"] for s in st) > 0 and sum(s["evicted"] for s in st) > 0
    assert not any(s["rebuilt"] for s in st)


def test_frames_with_visibility(setup, orc):
    csv, blobs, labels = setup
    run_frames(csv, orc, blobs, labels, 256 << 20, seed=5, density=0.002)


def test_frames_small_cache_rebuilds(setup, orc):
    csv, blobs, labels = setup
    # a little more than the largest frame needs: reuse from the stacks,
    # then rebuilds when fragmentation runs the top to the end
    st = run_frames(csv, orc, blobs, labels, 6912 << 10, n_frames=10, seed=7)
    assert any(s["rebuilt"] for s in st)


def test_frames_mixed_rebuilds_and_overflows(setup, orc):
    csv, blobs, labels = setup
    # frames that alone exceed the cache fail (nothing cached); the next
    # frames start from an empty cache
    st = run_frames(csv, orc, blobs, labels, 6400 << 10, n_frames=10, seed=7, expect_error=True)
    assert any(s["rebuilt"] for s in st) and len(st) < 10


@pytest.mark.parametrize("cap,n_frames,seed,density,err", [(256 << 20, 8, 5, 0.002, False), (6912 << 10, 10, 7, None, False),
                                                       (6400 << 10, 10, 7, None, True)])
def test_frames_without_stats(setup, orc, cap, n_frames, seed, density, err):
    # the same frames with the decode's count read on the device: same
    # blocks, same counts (read afterwards), rebuilds and overflows included
    csv, blobs, labels = setup
    st = run_frames(csv, orc, blobs, labels, cap, n_frames=n_frames, seed=seed, density=density, expect_error=err,
                    sync=False)
    assert st


def test_frame_graph_replays(setup, orc):
    # a frame without statistics captured in a graph and replayed for new
    # request lists, each replay checked against the same frame run eagerly
    # on a second cache (with eager work and synchronisation in between)
    csv, blobs, labels = setup
    torch = torch_cuda()
    pool = csv.Pool()
    for b in blobs:
        pool.add_volume(b)
    nb = len(labels)
    seq = frames(nb, 5, seed=11)
    s = torch.cuda.Stream()
    eager = csv.FrameCache(pool, 64 << 20, 512)
    graph = csv.FrameCache(pool, 64 << 20, 512)
    ids_g = torch.from_numpy(seq[0][0].view(np.int32)).cuda()
    lods_g = torch.from_numpy(seq[0][1]).cuda()
    slots_g = torch.empty(len(seq[0][0]), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        # the first frame outside the capture sizes the stream's buffers
        log("graph: frame 1 eager on both caches")
        graph.frame(ids_g, lods_g, slots=slots_g, stream=s, stats=False)
        eager.frame(ids_g, lods_g, stream=s, stats=False)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        graph.frame(ids_g, lods_g, slots=slots_g, stream=s, stats=False)
    for f in range(1, 5):
        ids, lods = seq[f]
        ids_g.copy_(torch.from_numpy(ids.view(np.int32)))
        lods_g.copy_(torch.from_numpy(lods))
        torch.cuda.synchronize()
        log("graph: replay for frame %d" % (f + 1))
        g.replay()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            slots_e, _ = eager.frame(ids_g.clone(), lods_g.clone(), stream=s, stats=False)
        s.synchronize()
        # block positions depend on the order in which the mark kernel's
        # atomics list the misses, so the two caches agree on what is stored
        # and on the counts, and each block holds its brick
        sg, se = slots_g.cpu().numpy(), slots_e.cpu().numpy()
        np.testing.assert_array_equal(sg >= 0, se >= 0)
        st_g, st_e = graph.last_stats(), eager.last_stats()
        assert st_g == st_e and st_g["frame"] == f + 1
        for i, t, sl, sl_e in zip(ids.tolist(), lods.tolist(), sg.tolist(), se.tolist()):
            if sl >= 0:
                n = (32 >> t) ** 3
                ref = decode_ref(orc, blobs, int(i), int(t))
                np.testing.assert_array_equal(graph.read(sl, n), ref)
                np.testing.assert_array_equal(eager.read(sl_e, n), ref)
    del g
    graph.close()
    eager.close()


def test_frame_larger_than_cache(setup, orc):
    csv, blobs, labels = setup
    run_frames(csv, orc, blobs, labels, 256 << 10, n_frames=2, seed=9, expect_error=True)


def test_empty_frame_and_bad_arguments(setup):
    csv, blobs, labels = setup
    torch = torch_cuda()
    pool = csv.Pool()
    pool.add_volume(blobs[0])
    cache = csv.FrameCache(pool, 1 << 20, 16)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    slots, st = cache.frame(e, e.to(torch.uint8))
    assert st["distinct"] == 0 and st["frame"] == 1
    too_many = torch.zeros(17, dtype=torch.int32, device="cuda")
    with pytest.raises(csv.CsvError):
        cache.frame(too_many, too_many.to(torch.uint8))
    with pytest.raises(csv.CsvError):
        cache.read(1 << 30, 8)
