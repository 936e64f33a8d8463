"""GPU: detail streaming in frames (Sec. 4.2) on the frame cache.  A pool
keeps level-0 detail in pinned host memory; a camera moves through a 256^3
cut of the cells volume and each frame requests every brick at the level
of detail its distance gives.  A full-LOD request whose detail is not on
the device is served at LOD 1 (the paper's first option) and its detail is
uploaded for the next frame; with predictions (the bricks close to the
camera, the paper's second option) the detail arrives before the first
full-LOD request.

Expectations: every served block equals the oracle's decode of its brick at
the served LOD; which requests are served at LOD 1, and the frame's detail
counts, equal a host model of the policy (staging in order until the
buffer is full, detail kept while the new detail fits behind it, dropped
otherwise); the decoder never takes its own level-1 fallback (the pool's
error word stays clear)."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

G = 8          # bricks per axis (256^3 voxels)
D0 = 80.0      # full LOD within 80 voxels of the camera
STEP = 24.0    # camera travel per frame (voxels)


def log(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup(orc):
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    vol = synth.cells(n=512, grid=37, seed=2)[:256, :256, :256].copy()
    blob = orc.encode_volume(vol, scale_bits=10, lane_k=64)
    labels = [np.unique(vol[32 * bz:32 * bz + 32, 32 * by:32 * by + 32, 32 * bx:32 * bx + 32])
              for bz in range(G) for by in range(G) for bx in range(G)]
    return csv, blob, {}, labels


def detail_pool(csv, blob, staging=None):
    pool = csv.Pool()
    assert pool.add_volume(blob, detail_host=True) == 0
    if staging is not None:
        pool.set_detail_staging(staging)
    gran = np.array([pool.detail_bytes(i) for i in range(G ** 3)], np.int64)
    assert (gran > 0).sum() > G ** 3 // 2
    return pool, gran


def path(n_frames):
    """Camera positions along x through the middle of the volume."""
    return [(-40.0 + STEP * k, 120.0, 136.0) for k in range(n_frames)]


class Model:
    """Host model of which full-LOD requests are served at LOD 1 and of the
    staging of detail between frames."""

    def __init__(self, gran, cap):
        self.gran, self.cap = gran, cap
        self.staged, self.used = set(), 0
        self.cached0 = set()   # bricks whose full LOD is cached after the last frame
        self.want, self.pred = [], []

    def frame(self, ids, lods, predict, vis=None, cap_bytes=None):
        """vis: per request visible (None: all); cap_bytes: cache size (a
        frame whose distinct blocks exceed it stores nothing).  Returns the
        served LODs (0xFF: not stored), the detail counts and whether the
        frame did not fit."""
        if vis is None:
            vis = np.ones(len(ids), bool)
        lst = list(dict.fromkeys(sorted(self.want) + list(self.pred)))
        fresh = [b for b in lst if b not in self.staged]
        need = sum(int(self.gran[b]) for b in fresh)
        released = 0
        if self.staged and self.used + need > self.cap:
            self.staged, self.used, released = set(), 0, 1
            fresh = lst
        up = 0
        for b in fresh:
            if self.used + int(self.gran[b]) > self.cap:
                break
            self.staged.add(b)
            self.used += int(self.gran[b])
            up += int(self.gran[b])
        ds = dict(wanted=len(self.want), predicted=len(self.pred), staged=sum(b in self.staged for b in lst),
                  released=released, uploaded_bytes=up, resident_bytes=self.used)
        served = np.where(vis & (lods < 5), lods, 0xFF).astype(np.uint8)
        fb = set()
        for r, (b, t) in enumerate(zip(ids.tolist(), served.tolist())):
            if t == 0 and self.gran[b] and b not in self.cached0 and b not in self.staged:
                served[r] = 1
                fb.add(b)
        ds["fallbacks"] = len(fb)
        keys = {(b, t) for b, t in zip(ids.tolist(), served.tolist()) if t != 0xFF}
        error = cap_bytes is not None and sum(32 << (3 * (4 - t)) for _, t in keys) > cap_bytes
        if error:
            served[:] = 0xFF
        self.cached0 = {b for b, t in keys if t == 0 and not error}
        self.want = sorted(fb)
        self.pred = [int(b) for b in predict if self.gran[b] and int(b) not in self.cached0]
        return served, ds, error


def run(csv, orc, blob, refs, n_frames, radius=None, staging=None, stats=True, check_all=True, cache_bytes=256 << 20,
        density=None, labels=None):
    """Frames along the path; radius: predict the bricks within that many
    voxels; density: a share of the labels visible (a new draw every other
    frame; labels: each brick's labels).  Returns per frame (served LODs,
    detail stats or None for a frame that did not fit)."""
    pool, gran = detail_pool(csv, blob, staging)
    cap = staging if staging is not None else 8 << 20
    cache = csv.FrameCache(pool, cache_bytes, G ** 3)
    model = Model(gran, cap)
    out = []
    try:
        frames_along(csv, orc, blob, refs, n_frames, radius, stats, check_all, pool, cache, model, out, cache_bytes,
                     density, labels)
    finally:
        cache.close()
    return out


def frames_along(csv, orc, blob, refs, n_frames, radius, stats, check_all, pool, cache, model, out, cache_bytes,
                 density, labels):
    torch = torch_cuda()
    for k, pos in enumerate(path(n_frames)):
        ids, lods = synth.frame_requests(G, G, G, pos, D0)
        pred = synth.near_bricks(G, G, G, pos, radius) if radius else np.zeros(0, np.uint32)
        vis, bits, n_lab = None, None, 0
        if density is not None and k % 2 == 1:
            n_lab = int(max(l.max() for l in labels)) + 1
            show = np.random.default_rng(200 + k).random(n_lab) < density
            words = np.zeros((n_lab + 31) // 32, np.uint32)
            idx = np.nonzero(show)[0].astype(np.uint64)
            np.bitwise_or.at(words, (idx >> 5).astype(np.int64),
                             (np.uint64(1) << (idx & np.uint64(31))).astype(np.uint32))
            bits = torch.from_numpy(words.view(np.int32)).cuda()
            vis = np.array([bool(show[labels[i]].any()) for i in ids])
        want_served, want_ds, error = model.frame(ids, lods, pred, vis, cache_bytes)
        log("frame %d at x=%.0f: %d full-LOD requests, %d predicted, %s visible, stats %s, %s"
            % (k + 1, pos[0], int((lods == 0).sum()), len(pred), "all" if vis is None else int(vis.sum()), stats,
               "does not fit" if error else "fits"))
        d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
        d_lods = torch.from_numpy(lods).cuda()
        d_pred = torch.from_numpy(pred.view(np.int32)).cuda() if len(pred) else None
        slots = torch.empty(len(ids), dtype=torch.int64, device="cuda")
        served = torch.empty(len(ids), dtype=torch.uint8, device="cuda")
        st = ds = None
        if error and stats:
            with pytest.raises(csv.CsvError) as e:
                cache.frame_detail(d_ids, d_lods, predict=d_pred, visible_bits=bits, n_label_bits=n_lab,
                                   slots=slots, served=served)
            assert e.value.code == csv.CSV_ENOMEM
        else:
            _, _, st, ds = cache.frame_detail(d_ids, d_lods, predict=d_pred, visible_bits=bits, n_label_bits=n_lab,
                                              slots=slots, served=served, stats=stats)
        torch.cuda.synchronize()
        assert pool.last_error() == (0, 0)
        served = served.cpu().numpy()
        slots = slots.cpu().numpy()
        np.testing.assert_array_equal(served, want_served)
        if error:
            assert (slots == -1).all()
            if not stats:
                with pytest.raises(csv.CsvError):
                    cache.last_stats()
            out.append((served, None))
            continue
        if stats:
            assert ds == want_ds, (k, ds, want_ds)
            assert st["frame"] == k + 1
        else:
            assert st is None and ds is None
        if check_all or k in (0, n_frames - 1):
            used = cache.last_stats()["used_bytes"] // 4
            data = cache.read(0, used)
            for i, t, s in zip(ids.tolist(), served.tolist(), slots.tolist()):
                if t == 0xFF:
                    assert s == -1
                    continue
                if (i, t) not in refs:
                    refs[(i, t)] = orc.decode_brick(blob, i, t).ravel()
                g = 32 >> t
                np.testing.assert_array_equal(data[s:s + g ** 3], refs[(i, t)], err_msg="brick %d lod %d" % (i, t))
        out.append((served, ds))


def test_without_prediction_a_fallback_lasts_one_frame(setup, orc):
    csv, blob, refs, _ = setup
    res = run(csv, orc, blob, refs, 12)
    fbs = [ds["fallbacks"] for _, ds in res]
    log("fallbacks per frame %s" % fbs)
    assert fbs[0] > 0 and sum(fbs[1:]) > 0
    # a brick served at LOD 1 for want of detail is served at full LOD by the next frame that asks for it
    for k in range(len(res) - 1):
        ids, lods = synth.frame_requests(G, G, G, path(12)[k], D0)
        ids2, lods2 = synth.frame_requests(G, G, G, path(12)[k + 1], D0)
        fell = set(ids[(lods == 0) & (res[k][0] == 1)].tolist())
        again = (lods2 == 0) & np.isin(ids2, list(fell))
        assert (res[k + 1][0][again] == 0).all()


def test_prediction_hides_the_lag(setup, orc):
    csv, blob, refs, _ = setup
    res = run(csv, orc, blob, refs, 12, radius=D0 + 2 * STEP)
    fbs = [ds["fallbacks"] for _, ds in res]
    log("fallbacks per frame with prediction %s" % fbs)
    assert fbs[0] > 0 and sum(fbs[1:]) == 0
    assert all(ds["predicted"] > 0 for _, ds in res[1:])


def test_small_staging_buffer(setup, orc):
    csv, blob, refs, _ = setup
    res = run(csv, orc, blob, refs, 10, radius=D0 + 2 * STEP, staging=16 << 10)
    log("detail stats %s" % [ds for _, ds in res])
    assert sum(ds["released"] for _, ds in res) > 0
    assert sum(ds["fallbacks"] for _, ds in res[1:]) > 0


@pytest.mark.parametrize("cache_mib,radius", [(256, None), (22, D0 + STEP), (12, None), (12, D0 + STEP)])
def test_visibility_rebuilds_and_frames_too_large(setup, orc, cache_mib, radius):
    # invisible requests are not stored and want no detail; a cache a little
    # larger than a frame rebuilds; frames larger than the cache store
    # nothing, and their fallbacks are still listed for the next frame
    csv, blob, refs, labels = setup
    res = run(csv, orc, blob, refs, 10, radius=radius, cache_bytes=cache_mib << 20, density=0.02, labels=labels)
    if cache_mib == 12:
        assert any(ds is None for _, ds in res)


def test_frames_without_statistics_serve_the_same(setup, orc):
    csv, blob, refs, _ = setup
    a = run(csv, orc, blob, refs, 8, radius=D0 + STEP, check_all=False)
    b = run(csv, orc, blob, refs, 8, radius=D0 + STEP, stats=False, check_all=False)
    for (sa, _), (sb, _) in zip(a, b):
        np.testing.assert_array_equal(sa, sb)


def test_plain_frames_refused_and_pools_without_detail(setup, orc):
    csv, blob, refs, _ = setup
    torch = torch_cuda()
    pool, _ = detail_pool(csv, blob)
    cache = csv.FrameCache(pool, 64 << 20, 64)
    ids = torch.arange(8, dtype=torch.int32, device="cuda")
    lods = torch.zeros(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(csv.CsvError) as e:
        cache.frame(ids, lods)
    assert e.value.code == csv.CSV_EINVAL
    cache.close()
    # on a pool whose records are whole in HBM every request is served at its own LOD
    whole = csv.Pool()
    whole.add_volume(blob)
    cache = csv.FrameCache(whole, 64 << 20, 64)
    lods = torch.tensor([0, 1, 2, 5, 0, 0, 3, 4], dtype=torch.uint8, device="cuda")
    pred = torch.arange(4, dtype=torch.int32, device="cuda")
    slots, served, st, ds = cache.frame_detail(ids, lods, predict=pred)
    assert served.cpu().tolist() == [0, 1, 2, 0xFF, 0, 0, 3, 4]
    assert ds["fallbacks"] == 0 and ds["wanted"] == 0 and st["decoded"] == 7
    data = cache.read(0, st["used_bytes"] // 4)
    for i, (t, s) in enumerate(zip(served.cpu().tolist(), slots.cpu().tolist())):
        if t != 0xFF:
            np.testing.assert_array_equal(data[s:s + (32 >> t) ** 3], orc.decode_brick(blob, i, t).ravel())
    cache.close()
