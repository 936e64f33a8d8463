#!/usr/bin/env python3
"""Benchmark: GPU decode throughput of compressed segmentation volumes.

Workload (one step): decode all 32,768 bricks of a 1024^3 uint32
neurite-like volume (20,000 labels, random-walk branching tubes of radius
2-8 voxels, Zipf-distributed sizes, about 45 % background; seeded synthetic
data) at full level of detail in one decode call of the HIP decoder, the
compressed pool and the 4.3 GB output resident in HBM.

Prints one JSON line: decoded GB/s (uint32 labels), the HBM roofline of the
decode call, the same volume at half LOD, 16,384 uneven mixed-LOD requests
over three volumes, a 512^3 cells volume, the one-launch-per-brick
baseline, the CPU oracle (all host threads and one), detail separation,
the GPU compressor and the serving loop.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM bytes of one decode call on the headline workload (front + leaf
# kernel), from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by
# what the same counters read for a plain 256 MiB device copy; see
# profiles/decode_neurite1024_hbm_traffic.md.  Valid only for the decoder
# source the counters were taken on (at the launch shape named here).
TRAFFIC = {"decoder_sha256_16": "200266273e9e1f32", "shape": (8, 3, 0, 0, 4), "bytes": 5094037997}
PAPER_GBS = {"cells": 9.9, "fiber": 10.4, "cortex": 9.3}  # Table 3, RTX 3070 Ti (context only)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def decoder_hash():
    """sha256 prefix of the decoder's sources (kernels and the table format)."""
    h = hashlib.sha256()
    for f in ("csv_decode.hip", "csv_format.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2308_16619_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def record_sizes(blob: bytes) -> np.ndarray:
    B = int(np.frombuffer(blob, np.uint32, 1, 36)[0])
    idx = np.frombuffer(blob, np.uint64, B + 1, 128)
    return np.diff(idx).astype(np.int64)


def record_bytes(blob: bytes, ids) -> int:
    """Compressed bytes a full-LOD decode of `ids` must read: each whole
    record (header, palette, lane states, all words)."""
    return int(record_sizes(blob)[np.asarray(ids)].sum())


def prefix_record_bytes(csv, blob: bytes) -> tuple:
    """Per brick, the bytes a decode to level 1 must read: header, palette,
    lane states and the words of the level-1 prefix (rounded up to a dword).
    The pool's detail separation finds that prefix (it decodes every brick to
    level 1 once and keeps exactly those bytes on the device); a brick whose
    record is all prefix keeps its whole record."""
    p = csv.Pool(0)
    p.add_volume(blob, detail_host=True)
    sizes = record_sizes(blob)
    host = p.info()["host_bytes"]
    p.close()
    return sizes, int(sizes.sum()) - int(host)


def timed_calls(torch, fn, steps, warmup):
    """ms per call of fn() over `steps` calls (HIP events on the current stream)."""
    for _ in range(warmup):
        fn()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def frame_cache_leg(csv, torch, pool, ids, lods, t_ns, fps=60):
    """Frame cache (Sec. 4.1) on the same pool: the trace cut into frames of
    1/fps s; per frame one call (mark, evict, assign, decode of the new
    bricks), timed from the call to the end of its decode."""
    f = (t_ns // int(1e9 / fps)).astype(np.int64)
    nf = int(f.max()) + 1
    bounds = np.searchsorted(f, np.arange(nf + 1))
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_lods = torch.from_numpy(lods).cuda()
    max_req = int(np.diff(bounds).max())
    slots = torch.empty(max_req, dtype=torch.int64, device="cuda")
    runs = []
    # 16 GiB holds any frame; 1.5 GiB is about one frame's bricks (rebuilds, and
    # frames too large for the cache, which then holds nothing)
    for cache_gib in (16, 1.5):
        fc = csv.FrameCache(pool, int(cache_gib * 2 ** 30), max_req)
        ms, sts, overflow = [], [], 0
        for k in range(nf):
            a, b = int(bounds[k]), int(bounds[k + 1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                _, st = fc.frame(d_ids[a:b], d_lods[a:b], slots=slots[:b - a])
            except csv.CsvError as e:
                if e.code != csv.CSV_ENOMEM:
                    raise
                overflow += 1
                st = {"distinct": 0, "decoded": 0, "hits": 0, "rebuilt": 1, "used_bytes": 0}
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            sts.append(st)
        fc.close()
        assert pool.last_error()[0] == 0
        ms_s = sorted(ms[1:])  # the first frame fills an empty cache
        dist = sum(s["distinct"] for s in sts[1:])
        runs.append({"cache_gib": cache_gib, "frames": nf, "first_frame_ms": round(ms[0], 3),
                     "p50_ms": round(ms_s[len(ms_s) // 2], 3), "p99_ms": round(ms_s[int(0.99 * (len(ms_s) - 1))], 3),
                     "max_ms": round(ms_s[-1], 3),
                     "distinct_per_frame": round(dist / max(nf - 1, 1), 1),
                     "decoded_per_frame": round(sum(s["decoded"] for s in sts[1:]) / max(nf - 1, 1), 1),
                     "hit_rate": round(sum(s["hits"] for s in sts[1:]) / max(dist, 1), 4),
                     "rebuilds": sum(s["rebuilt"] for s in sts), "frames_too_large": overflow,
                     "used_gib": round(sts[-1]["used_bytes"] / 2 ** 30, 3)})
        log("frame cache %s" % runs[-1])
    # the same frames in a 16 GiB cache without statistics: no host round
    # trip (the decode takes its count from device memory)
    fc = csv.FrameCache(pool, 16 << 30, max_req)
    ms = []
    for k in range(nf):
        a, b = int(bounds[k]), int(bounds[k + 1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fc.frame(d_ids[a:b], d_lods[a:b], slots=slots[:b - a], stats=False)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    last = fc.last_stats()
    fc.close()
    assert pool.last_error()[0] == 0
    ms_s = sorted(ms[1:])
    no_stats = {"cache_gib": 16, "frames": nf, "last_frame": last["frame"], "p50_ms": round(ms_s[len(ms_s) // 2], 3),
                "p99_ms": round(ms_s[int(0.99 * (len(ms_s) - 1))], 3), "max_ms": round(ms_s[-1], 3)}
    log("frame cache without statistics %s" % no_stats)
    return {"fps": fps, "requests_per_frame": round(len(ids) / nf, 1), "runs": runs, "without_stats": no_stats}


def serving_leg(csv, synth, seconds):
    """Serving: the 2048x2048x1024 neurite volume (131,072 bricks, 80,000
    labels) resident in HBM as a compressed pool; brick requests of a camera
    fly-through (Poisson arrivals, view-cone sampling, LOD by distance)
    replayed in real time at 1M and 5M requests/s, with a decoded-brick
    cache of 16 GiB (holds every brick) and of 2 GiB (forces eviction).
    0.2 s of warm-up requests precede the measured `seconds`."""
    nx, ny, nz = 2048, 2048, 1024
    log("serving: generating the %dx%dx%d neurite volume" % (nx, ny, nz))
    t0 = time.time()
    vol = synth.neurite(nx, ny, nz, labels=80000, seed=8)
    log("generated in %.1fs; encoding" % (time.time() - t0))
    blob = csv.encode_volume(vol)
    raw = vol.nbytes
    del vol
    pool = csv.Pool(0)
    pool.add_volume(blob)
    if os.path.exists(csv.TUNING_PATH):
        pool.load_tuning()
    log("pool: %d bytes compressed (%.3f%% of %d)" % (len(blob), 100.0 * len(blob) / raw, raw))
    runs = []
    for rate in (1e6, 5e6):
        wi, wl, wt = synth.camera_trace(nx, ny, nz, rate, 0.2, seed=16, t0_s=0.0)
        mi, ml, mt = synth.camera_trace(nx, ny, nz, rate, seconds, seed=26, t0_s=0.2)
        warm = csv.Server.requests(wi, wl, t_arrival_ns=wt)
        main = csv.Server.requests(mi, ml, t_arrival_ns=mt)
        hist = np.bincount(ml, minlength=3)[:3] / max(len(ml), 1)
        for cache_gib in (16, 2):
            srv = csv.Server(pool, cache_bytes=cache_gib << 30, inflight_bytes=1 << 30, max_batch=4096, streams=4)
            srv.run_trace(warm, timeout_s=30)
            srv.reset_stats()
            _, got = srv.run_trace(main, timeout_s=60)
            st = srv.stats()
            srv.close()
            r = {"offered_per_s": rate, "cache_gib": cache_gib, "requests": int(len(main)), "completed": int(got),
                 "completed_per_s": round(got / seconds, 1), "p50_us": round(st["p50_us"], 1),
                 "p99_us": round(st["p99_us"], 1), "p99_miss_us": round(st["p99_miss_us"], 1),
                 "max_us": round(st["max_us"], 1),
                 "hit_rate": round(st["hits"] / max(st["requests"], 1), 4),
                 "p50_miss_us": round(st["p50_miss_us"], 1),
                 "joined": int(st["joined"]), "evictions": int(st["evictions"]), "rebuilds": int(st["rebuilds"]),
                 "batches": int(st["batches"]), "mean_batch": round(st["misses"] / max(st["batches"], 1), 1),
                 "stalls_batch_inflight_slot": [int(st["stall_batch"]), int(st["stall_inflight"]),
                                                int(st["stall_slot"])],
                 "decoded_gb": round(st["decoded_bytes"] / 1e9, 3),
                 "worker_busy_frac": round(st["worker_busy_ns"] * 1e-9 / seconds, 3),
                 "worker_launch_frac": round(st["worker_launch_ns"] * 1e-9 / seconds, 3),
                 "lod_hist": [round(float(x), 4) for x in hist]}
            log("serving %s" % r)
            runs.append(r)
    # detail separation (Sec. 4.2): the same volume with level-0 detail in
    # host memory, served at 1M/s with the 16 GiB cache (full-LOD misses
    # stage their detail through the pool's 8 MiB buffer, batch by batch)
    dpool = csv.Pool(0)
    dpool.add_volume(blob, detail_host=True)
    wi, wl, wt = synth.camera_trace(nx, ny, nz, 1e6, 0.2, seed=16, t0_s=0.0)
    mi, ml, mt = synth.camera_trace(nx, ny, nz, 1e6, seconds, seed=26, t0_s=0.2)
    srv = csv.Server(dpool, cache_bytes=16 << 30, inflight_bytes=1 << 30, max_batch=4096, streams=4)
    srv.run_trace(csv.Server.requests(wi, wl, t_arrival_ns=wt), timeout_s=30)
    srv.reset_stats()
    _, got = srv.run_trace(csv.Server.requests(mi, ml, t_arrival_ns=mt), timeout_s=60)
    st = srv.stats()
    srv.close()
    di = dpool.info()
    detail = {"offered_per_s": 1e6, "cache_gib": 16, "requests": int(len(mi)), "completed": int(got),
              "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1),
              "p99_miss_us": round(st["p99_miss_us"], 1), "hit_rate": round(st["hits"] / max(st["requests"], 1), 4),
              "host_detail_bytes": int(di["host_bytes"]), "staged_bytes": int(st["detail_staged_bytes"]),
              "releases": int(st["detail_releases"]), "stall_staging": int(st["stall_staging"]),
              "error": int(st["error"])}
    log("serving with detail in host memory %s" % detail)
    del dpool
    import torch
    mi, ml, mt = synth.camera_trace(nx, ny, nz, 1e6, seconds, seed=26, t0_s=0.0)
    frames = frame_cache_leg(csv, torch, pool, mi, ml, mt)
    worst = max(r["p99_us"] for r in runs)
    # the stated configuration is the 16 GiB cache; the 2 GiB cache is a stress case
    stated = max(r["p99_us"] for r in runs if r["cache_gib"] == 16)
    return {"workload": "2048x2048x1024 neurite (131,072 bricks, 80,000 labels), camera-path Poisson traces",
            "p99_us_16gib_cache": stated, "p99_us_worst": worst, "runs": runs,
            "frame_cache": frames, "detail_host": detail}


def detail_leg(csv, torch, blob, ids_np, ids, out, shape, whole_pool, reps=10):
    """Detail separation (Sec. 4.2) on the same volume: a second pool keeps in
    HBM only each record's level-1 prefix and the level-0 detail in pinned
    host memory.  A frame stages the detail of the requested bricks through
    the staging buffer (8 MiB, as in the paper) and decodes them at full LOD;
    its output must equal the whole-record pool's."""
    B = len(ids_np)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    dpool = csv.Pool(0)
    dpool.add_volume(blob, detail_host=True)
    add_s = time.perf_counter() - t0
    dpool.set_shape(shape)
    host = dpool.info()["host_bytes"]
    rec = csv.blob_info(blob)["record_bytes"]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def timed(pool, o, lod, n=10):
        pool.decode(ids, o, lod=lod)
        ev[0].record(stream)
        for _ in range(n):
            pool.decode(ids, o, lod=lod)
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / n

    # level 1 of every brick from the device prefix alone
    o1 = torch.empty(B * 16 ** 3, dtype=torch.int32, device=out.device)
    w1 = torch.empty_like(o1)
    whole_ms = timed(whole_pool, w1, 1)
    split_ms = timed(dpool, o1, 1)
    assert dpool.last_error()[0] == 0 and whole_pool.last_error()[0] == 0
    assert torch.equal(o1, w1), "level 1 of the split pool differs"
    del o1, w1
    # frames: stage, decode at full LOD, release; the reference is the
    # whole-record pool's decode, taken here (the caller's buffer is shared
    # with other legs)
    whole_pool.decode(ids, out, lod=0)
    out2 = torch.empty_like(out)
    st, dec, wall, done = [], [], [], 0
    for r in range(reps + 2):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev[0].record(stream)
        done = dpool.stage_detail(ids_np, stream)
        ev[1].record(stream)
        dpool.decode(ids[:done], out2, lod=0)
        ev[2].record(stream)
        dpool.release_detail(stream)
        torch.cuda.synchronize()
        if r >= 2:
            wall.append((time.perf_counter() - w0) * 1e3)
            st.append(ev[0].elapsed_time(ev[1]))
            dec.append(ev[1].elapsed_time(ev[2]))
    assert dpool.last_error()[0] == 0
    n_el = done * 32 ** 3
    assert torch.equal(out2[:n_el], out[:n_el]), "staged full-LOD decode differs"
    # full LOD with nothing staged: level 1 upsampled, CSV_EDETAIL recorded
    fb_ms = timed(dpool, out2, 0)
    assert dpool.last_error()[0] == csv.CSV_EDETAIL
    del out2
    cam = camera_frames(csv, torch, dpool, csv.blob_info(blob))
    med = lambda v: sorted(v)[len(v) // 2]
    staged_bytes = host if done == B else None
    return {"record_bytes": rec, "hbm_record_bytes": rec - host, "host_detail_bytes": host,
            "detail_frac": round(host / rec, 4), "add_volume_s": round(add_s, 3),
            "lod1_ms_split": round(split_ms, 4), "lod1_ms_whole": round(whole_ms, 4),
            "frame": {"bricks": done, "staging_bytes": 8 << 20, "detail_bytes": staged_bytes,
                      "stage_ms": round(med(st), 4), "decode_ms": round(med(dec), 4),
                      "wall_ms": round(med(wall), 4),
                      "stage_gbs": round(staged_bytes / (med(st) * 1e-3) / 1e9, 2) if staged_bytes else None},
            "unstaged_full_lod_ms": round(fb_ms, 4), "camera_frames": cam}


def camera_frames(csv, torch, dpool, info, n_frames=60, step=8.0, d0=96.0, ahead=4):
    """Detail streaming in frames (Sec. 4.2) on the pool with level-0 detail
    in host memory: a camera moves `step` voxels per frame along x through
    the middle of the volume; each frame requests every brick at the level
    of detail its distance gives (full LOD within d0 voxels) through the
    frame cache.  Without prediction a brick entering the full-LOD zone is
    served at LOD 1 for one frame; with prediction the detail of the bricks
    within d0 + ahead * step voxels is uploaded one frame ahead.  Per-frame
    wall time from the call to the end of its decode."""
    import synth
    g = info["nbx"], info["nby"], info["nbz"]
    runs = {}
    for mode, radius in (("on_demand", None), ("predictive", d0 + ahead * step)):
        fc = csv.FrameCache(dpool, 256 << 20, g[0] * g[1] * g[2])
        ms, fbs, up, res = [], [], [], []
        for k in range(n_frames):
            pos = (-40.0 + step * k, info["ny"] / 2 - 6, info["nz"] / 2 + 6)
            ids, lods = synth.frame_requests(*g, pos, d0)
            d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
            d_lods = torch.from_numpy(lods).cuda()
            pred = None
            if radius:
                pred = torch.from_numpy(synth.near_bricks(*g, pos, radius).view(np.int32)).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st, ds = fc.frame_detail(d_ids, d_lods, predict=pred)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            fbs.append(ds["fallbacks"])
            up.append(ds["uploaded_bytes"])
            res.append(ds["resident_bytes"])
        fc.close()
        dpool.release_detail()
        assert dpool.last_error()[0] == 0
        ms_s = sorted(ms[1:])  # the first frame fills an empty cache
        runs[mode] = {"frames": n_frames, "p50_ms": round(ms_s[len(ms_s) // 2], 3),
                      "p99_ms": round(ms_s[int(0.99 * (len(ms_s) - 1))], 3),
                      "first_frame_fallbacks": fbs[0],
                      "fallbacks_after_first": int(sum(fbs[1:])),
                      "frames_with_fallbacks": int(sum(1 for f in fbs[1:] if f)),
                      "uploaded_kib_per_frame": round(sum(up[1:]) / max(n_frames - 1, 1) / 1024, 1),
                      "max_resident_kib": round(max(res) / 1024, 1)}
        log("camera frames %s %s" % (mode, runs[mode]))
    return {"step_voxels": step, "full_lod_voxels": d0, "predict_radius_voxels": d0 + ahead * step,
            "staging_bytes": 8 << 20, **runs}


def encoder_leg(csv, torch, vol, blob, host_s, host_threads, reps=3):
    """GPU compression of the volume (labels resident in HBM; the call returns
    with the container in host memory), checked byte for byte against the
    host compressor's container, which was timed when the volume was encoded."""
    d = torch.from_numpy(vol.view(np.int32)).to("cuda:0")
    torch.cuda.synchronize()
    got = csv.encode_volume_gpu(d)
    assert got == blob, "GPU container differs from the host compressor's"
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        csv.encode_volume_gpu(d)
        ts.append(time.perf_counter() - t0)
    s = sorted(ts)[len(ts) // 2]
    raw = vol.nbytes
    return {"gpu_ms": round(s * 1e3, 2), "gpu_gbs": round(raw / s / 1e9, 2), "host_ms": round(host_s * 1e3, 1),
            "host_gbs": round(raw / host_s / 1e9, 3), "host_threads": host_threads,
            "identical_bytes": True, "raw_bytes": raw, "compressed_bytes": len(blob)}


def write_tuning(pools, path):
    """One tuning file with the classes of several pools (later pools win)."""
    import tempfile
    head, lines = None, {}
    for p in pools:
        with tempfile.NamedTemporaryFile("r", suffix=".txt") as f:
            p.save_tuning(f.name)
            rows = open(f.name).read().splitlines()
        head = head or rows[0]
        for r in rows[1:]:
            lines[tuple(r.split()[:3])] = r
    with open(path, "w") as f:
        f.write("\n".join([head] + [lines[k] for k in sorted(lines)]) + "\n")


def config4_requests(n=16384, seed=5):
    """16,384 requests over three volumes (64^3 Voronoi, 512^3 cells, 512^3
    smooth blobs): source uniform, brick uniform within it, LOD uniform in
    {0, 1, 2}."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, 3, n)
    return rng, src


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="CPU oracle time on all host threads")
    ap.add_argument("--plain-bricks", type=int, default=1024, help="bricks in the per-brick-launch baseline")
    ap.add_argument("--legs", choices=["all", "headline"], default="all",
                    help="headline: only the timed full-LOD decode of the 1024^3 volume (for profiler runs)")
    ap.add_argument("--serving", choices=["full", "none"], default="full",
                    help="serving leg: the 2048x2048x1024 neurite pool with camera-path traces (full) or none")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="measured trace length per serving run")
    ap.add_argument("--detail", choices=["full", "none"], default="full",
                    help="detail-separation leg (the 512^3 cells volume with level-0 detail in host memory)")
    ap.add_argument("--encoder", choices=["full", "none"], default="full",
                    help="GPU compressor leg (the 512^3 cells volume compressed on the device)")
    ap.add_argument("--shape", default="", help="fixed launch shape 'waves,groups,queue,lpt,chunks' instead of the "
                                                 "tuned shapes")
    ap.add_argument("--retune", action="store_true",
                    help="sweep launch shapes on every workload instead of loading the shipped tuning file")
    ap.add_argument("--tuning-out", default="", help="write the tuned shapes of every workload to this file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this decoder runs on one GPU; --gpus %d is not supported (bricks are independent, "
              "so several GPUs would each decode their own share)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2308_16619_amd as csv

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda:0")
    csv.lib()
    headline_only = args.legs == "headline"
    fixed = tuple(int(v) for v in args.shape.split(",")) if args.shape else None

    tuned_pools = []

    def pick_shape(pool, ids, out, **kw):
        """The launch shape: fixed by --shape; else the shipped tuning file's
        shape for this request set's class (no sweep); else the autotuner's
        on this request set."""
        if fixed:
            pool.set_shape(fixed)
            return fixed, None
        if not args.retune and os.path.exists(csv.TUNING_PATH) and pool.load_tuning() > 0:
            shape, ms = pool.shape_for(int(ids.numel()), kw.get("lod", 0), kw.get("lods") is not None, with_ms=True)
            if ms > 0:  # a tuned class (the pool's untuned default has no time)
                return shape, "tuning file"
        shape, tune_ms = pool.autotune(ids, out, reps=3, **kw)
        torch.cuda.synchronize()
        assert pool.last_error()[0] == 0
        tuned_pools.append(pool)
        return shape, tune_ms

    # ---- headline: the 1024^3 neurite volume, every brick at full LOD ----
    log("generating the 1024^3 neurite volume")
    t0 = time.time()
    vol3 = synth.neurite(1024, 1024, 1024, labels=20000, seed=3)
    log("generated in %.1fs; encoding" % (time.time() - t0))
    host_threads = 16
    t0 = time.perf_counter()
    blob3 = csv.encode_volume(vol3, threads=host_threads)
    enc3_s = time.perf_counter() - t0
    info3 = csv.blob_info(blob3)
    log("encoded in %.1fs: %d bytes, CR %.3f%%" % (enc3_s, len(blob3), 100.0 * len(blob3) / vol3.nbytes))
    B3 = info3["n_bricks"]
    pool3 = csv.Pool(0)
    pool3.add_volume(blob3)
    ids3_np = np.arange(B3, dtype=np.uint32)
    ids3 = torch.from_numpy(ids3_np.view(np.int32)).to(dev)
    elems3 = B3 * 32 ** 3
    out3 = torch.empty(elems3, dtype=torch.int32, device=dev)
    out3_bytes = elems3 * 4
    in3_bytes = record_bytes(blob3, ids3_np)
    shape3, tune3 = pick_shape(pool3, ids3, out3, lod=0)
    log("shape %s (autotuned: %s ms)" % (shape3, tune3))
    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        pool3.decode(ids3, out3, lod=0)
    torch.cuda.synchronize()
    code, who = pool3.last_error()
    assert code == 0, ("decode error", code, who)
    # spot check against the input volume (full LOD is lossless)
    got = out3.view(B3, 32, 32, 32)
    for bid in (0, 12345, 20000, B3 - 1):
        bx, by, bz = bid % 32, (bid // 32) % 32, bid // 1024
        ref = torch.from_numpy(vol3[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32].astype(np.int64))
        assert torch.equal(got[bid].cpu().to(torch.int64) & 0xFFFFFFFF, ref), bid
    del got

    log("timing %d steps" % args.steps)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        pool3.decode(ids3, out3, lod=0)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1) / args.steps
    gbs = out3_bytes / (ms * 1e-3) / 1e9
    code, who = pool3.last_error()
    assert code == 0, ("decode error", code, who)
    # one decode call (front + leaf kernel) per step: the event time per step
    achieved = (in3_bytes + out3_bytes) / (ms * 1e-3) / 1e9
    src_hash = decoder_hash()
    # counters taken on this decoder source at this launch shape, else none
    traffic = TRAFFIC["bytes"] if (src_hash == TRAFFIC["decoder_sha256_16"] and
                                   tuple(shape3) == tuple(TRAFFIC["shape"] or ())) else None
    del vol3

    extra = {}
    plain = visibility = detail = encoder = cpu = serving = None
    if not headline_only:
        # ---- the same volume at half LOD (16^3 per brick) ----
        out_h = torch.empty(B3 * 16 ** 3, dtype=torch.int32, device=dev)
        sh_h, _ = pick_shape(pool3, ids3, out_h, lod=1)
        ms_h = timed_calls(torch, lambda: pool3.decode(ids3, out_h, lod=1, shape=sh_h), args.steps, args.warmup)
        assert pool3.last_error()[0] == 0
        _, in_h = prefix_record_bytes(csv, blob3)
        ob_h = B3 * 16 ** 3 * 4
        extra["neurite1024_half_lod"] = {
            "bricks": B3, "lod": 1, "ms_per_call": round(ms_h, 4), "gbs": round(ob_h / (ms_h * 1e-3) / 1e9, 2),
            "voxels_per_s": round(B3 * 16 ** 3 / (ms_h * 1e-3), 1), "read_bytes": in_h, "write_bytes": ob_h,
            "frac": round((in_h + ob_h) / (ms_h * 1e-3) / 1e9 / HBM_PEAK_GBS, 5), "shape": list(sh_h)}
        log("half LOD %s" % extra["neurite1024_half_lod"])
        del out_h

        # ---- baseline: one launch per brick ----
        nb = min(args.plain_bricks, B3)
        pids = ids3[:nb].contiguous()
        pout = out3[:nb * 32 ** 3]
        plain_ms = timed_calls(torch, lambda: pool3.decode(pids, pout, lod=0, plain=True), 1, 1)
        assert pool3.last_error()[0] == 0
        plain = {"value": round(nb * 32 ** 3 * 4 / (plain_ms * 1e-3) / 1e9, 3), "unit": "GB/s", "bricks": nb,
                 "ms": round(plain_ms, 3)}

        # ---- empty-space test (Sec. 4) of the same requests: a transfer
        # function showing a seeded 1 in 200 of the labels ----
        n_lab = 20001
        show = np.random.default_rng(11).random(n_lab) < 0.005
        words = np.zeros((n_lab + 31) // 32, np.uint32)
        nzl = np.nonzero(show)[0].astype(np.uint64)
        np.bitwise_or.at(words, (nzl >> 5).astype(np.int64), (np.uint64(1) << (nzl & np.uint64(31))).astype(np.uint32))
        d_words = torch.from_numpy(words.view(np.int32)).to(dev)
        vmask = torch.empty(B3, dtype=torch.uint8, device=dev)
        vis_ms = timed_calls(torch, lambda: pool3.visible(ids3, d_words, n_lab, out=vmask), 20, 3)
        assert pool3.last_error()[0] == 0
        visibility = {"bricks": B3, "us_per_call": round(vis_ms * 1e3, 2),
                      "bricks_per_s": round(B3 / (vis_ms * 1e-3), 1),
                      "visible_frac": round(float(vmask.float().mean().item()), 4),
                      "transfer_function": "a seeded 1 in 200 of the 20,000 labels visible"}

        # ---- the 512^3 cells volume (full LOD, 4096 bricks) ----
        log("generating the 512^3 cells volume")
        vol2 = synth.cells(n=512, grid=37, p_noise=0.5, seed=2)
        t0 = time.perf_counter()
        blob2 = csv.encode_volume(vol2, threads=host_threads)
        enc2_s = time.perf_counter() - t0
        pool2 = csv.Pool(0)
        pool2.add_volume(blob2)
        B2 = 4096
        ids2_np = np.arange(B2, dtype=np.uint32)
        ids2 = torch.from_numpy(ids2_np.view(np.int32)).to(dev)
        out2 = out3[:B2 * 32 ** 3]
        sh2, _ = pick_shape(pool2, ids2, out2, lod=0)
        ms2 = timed_calls(torch, lambda: pool2.decode(ids2, out2, lod=0, shape=sh2), args.steps, args.warmup)
        assert pool2.last_error()[0] == 0
        in2 = record_bytes(blob2, ids2_np)
        ob2 = B2 * 32 ** 3 * 4
        extra["cells512_full_lod"] = {
            "bricks": B2, "lod": 0, "ms_per_call": round(ms2, 4), "gbs": round(ob2 / (ms2 * 1e-3) / 1e9, 2),
            "voxels_per_s": round(B2 * 32 ** 3 / (ms2 * 1e-3), 1), "read_bytes": in2, "write_bytes": ob2,
            "frac": round((in2 + ob2) / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 5), "shape": list(sh2),
            "compressed_bytes": len(blob2), "compression_ratio_pct": round(100.0 * len(blob2) / vol2.nbytes, 4)}
        log("cells %s" % extra["cells512_full_lod"])

        # ---- small batches of the same volume (full LOD): time per call with
        # the library's shape (the paired front kernel) and with one wave per brick ----
        small, rng_s = [], np.random.default_rng(11)
        for nb in (32, 128, 512, 1024):
            ids_s = torch.from_numpy(rng_s.permutation(B2)[:nb].astype(np.int32)).to(dev)
            o_a = out2[:nb * 32 ** 3]
            o_b = torch.empty_like(o_a)
            auto = pool2.shape_for(nb, 0, False)
            ms_a = timed_calls(torch, lambda: pool2.decode(ids_s, o_a, lod=0), args.steps, args.warmup)
            unpaired = (8, 3, 0, 0, 1)
            ms_b = timed_calls(torch, lambda: pool2.decode(ids_s, o_b, lod=0, shape=unpaired), args.steps, args.warmup)
            assert pool2.last_error()[0] == 0 and torch.equal(o_a, o_b), "small batch outputs differ"
            small.append({"bricks": nb, "ms_per_call": round(ms_a, 4), "shape": list(auto),
                          "one_wave_per_brick_ms": round(ms_b, 4), "one_wave_per_brick_shape": list(unpaired)})
            del o_b
        extra["cells512_small_batches"] = small
        log("small batches %s" % small)

        # ---- 16,384 uneven mixed-LOD requests over three volumes, one persistent launch ----
        log("mixed requests over three volumes")
        vol1 = synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1)
        volb = synth.blobs(n=512, sites=50, amp=24.0, seed=4)
        blobs4 = [csv.encode_volume(vol1), blob2, csv.encode_volume(volb, threads=host_threads)]
        del volb
        pool4 = csv.Pool(0)
        first = [pool4.add_volume(b) for b in blobs4]
        counts = [len(record_sizes(b)) for b in blobs4]
        rng, src = config4_requests()
        n4 = len(src)
        local = np.array([rng.integers(0, counts[k]) for k in src], dtype=np.uint32)
        ids4_np = (np.array(first, dtype=np.uint32)[src] + local).astype(np.uint32)
        lods4 = rng.integers(0, 3, n4).astype(np.uint8)
        off4, tot4 = csv.output_offsets(lods4)
        d_ids4 = torch.from_numpy(ids4_np.view(np.int32)).to(dev)
        d_lods4 = torch.from_numpy(lods4.copy()).to(dev)
        d_off4 = torch.from_numpy(off4.view(np.int64)).to(dev)
        out4 = out3[:tot4]
        sh4, tune4 = pick_shape(pool4, d_ids4, out4, lods=d_lods4, out_offsets=d_off4)
        ms4 = timed_calls(torch, lambda: pool4.decode(d_ids4, out4, lods=d_lods4, out_offsets=d_off4, shape=sh4),
                          args.steps, args.warmup)
        assert pool4.last_error()[0] == 0
        # reads: whole records at full LOD, the level-1 prefix at LODs 1 and 2 (an upper bound at LOD 2)
        full_rec = np.concatenate([record_sizes(b) for b in blobs4])
        pre_rec = []
        for b in blobs4:
            sizes, dev_bytes = prefix_record_bytes(csv, b)
            pre_rec.append(sizes * (dev_bytes / max(int(sizes.sum()), 1)))
        pre_rec = np.concatenate(pre_rec)
        in4 = int(np.where(lods4 == 0, full_rec[ids4_np], pre_rec[ids4_np]).sum())
        ob4 = tot4 * 4
        sizes4 = full_rec[ids4_np]
        extra["mixed_16384"] = {
            "requests": n4, "lod_counts": [int((lods4 == t).sum()) for t in range(3)],
            "record_bytes_min_max": [int(sizes4.min()), int(sizes4.max())], "ms_per_call": round(ms4, 4),
            "gbs": round(ob4 / (ms4 * 1e-3) / 1e9, 2), "voxels_per_s": round(tot4 / (ms4 * 1e-3), 1),
            "read_bytes": in4, "write_bytes": ob4,
            "frac": round((in4 + ob4) / (ms4 * 1e-3) / 1e9 / HBM_PEAK_GBS, 5), "shape": list(sh4),
            "autotune_ms": tune4}
        log("mixed %s" % extra["mixed_16384"])
        del pool4

        if args.detail == "full":
            log("detail separation leg")
            detail = detail_leg(csv, torch, blob2, ids2_np, ids2, out2, sh2, pool2)
        if args.encoder == "full":
            log("GPU compressor leg")
            encoder = encoder_leg(csv, torch, vol2, blob2, enc2_s, host_threads)
        del vol2

        if not args.no_cpu:
            import oracle
            oracle._load()
            runs = []
            n_all = oracle.num_threads()
            # the same workload's first 2048 bricks, whole passes until the time is up
            sample = ids3_np[:2048]
            lods0 = np.zeros(len(sample), np.uint8)
            for threads, secs in ((n_all, args.cpu_seconds), (1, args.cpu_seconds / 2)):
                oracle.set_threads(threads)
                log("CPU oracle on %d threads (~%.0fs)" % (threads, secs))
                reps, t0 = 0, time.perf_counter()
                while True:
                    oracle.decode_bricks(blob3, sample[:len(sample) if threads > 1 else 256],
                                         lods0[:len(sample) if threads > 1 else 256])
                    reps += 1
                    el = time.perf_counter() - t0
                    if el >= secs or reps >= 500:
                        break
                nbk = len(sample) if threads > 1 else 256
                runs.append({"threads": threads, "gbs": round(reps * nbk * 32768 * 4 / el / 1e9, 4),
                             "sample": "%d passes over bricks 0..%d of the 1024^3 volume at full LOD (%.1f s)" %
                                       (reps, nbk - 1, el)})
            oracle.set_threads(n_all)
            cpu = {"value": runs[0]["gbs"], "unit": "GB/s", "cores": runs[0]["threads"], "kind": "oracle",
                   "sample": runs[0]["sample"], "single_thread": runs[1], "host_cpu": cpu_model(),
                   "host_logical_cpus": os.cpu_count()}

        if args.serving == "full":
            serving = serving_leg(csv, synth, args.serve_seconds)

    res = {
        "metric": "decoded GB/s (uint32 labels) + % HBM roofline; p50/p99 brick latency",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "1024^3 uint32 neurite-like volume (20,000 labels, random-walk branching tubes of "
                               "radius 2-8, Zipf sizes, ~45% background), 32,768 bricks of 32^3 decoded at full "
                               "LOD in one decode call",
                   "bricks": B3, "lod": 0, "compressed_bytes": len(blob3),
                   "compression_ratio_pct": round(100.0 * len(blob3) / (elems3 * 4), 4)},
        "voxels_per_s": round(elems3 / (ms * 1e-3), 1),
        "wall_s": round(t_wall, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "traffic_shape": list(TRAFFIC["shape"]) if traffic is not None else None,
                     "traffic_unit": "bytes per decode call", "algorithmic_bytes_per_launch": in3_bytes + out3_bytes,
                     "kernel": "csv_decode_bricks: per chunk of requests front_kernel then leaf_kernel, "
                               "chunks alternating between two streams", "shape": list(shape3),
                     "decoder_sha256_16": src_hash},
        "paper_context": {"gbs": PAPER_GBS, "hardware": "NVIDIA RTX 3070 Ti (Table 3; decoded bytes)"},
        "extra_workloads": extra,
        "plain_per_brick_launch": plain,
        "visibility_test": visibility,
        "detail_separation": detail,
        "encoder": encoder,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    if args.tuning_out and tuned_pools:
        write_tuning(tuned_pools, args.tuning_out)
        log("tuned shapes written to %s" % args.tuning_out)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
