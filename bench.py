#!/usr/bin/env python3
"""Benchmark: GPU decode throughput of compressed segmentation volumes.

Workload (one step): decode all 4096 bricks of a 512^3 uint32 'cells'
volume (jittered-grid Voronoi of 50,653 labels with 1-voxel boundary
noise, seeded synthetic data) at full level of detail, in one launch of the
HIP decoder, compressed pool and output resident in HBM.

Prints one JSON line: decoded GB/s (uint32 labels), the HBM roofline of the
decode kernel, the one-launch-per-brick baseline and the CPU oracle.
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

# HBM bytes of one decode call on this workload (front + leaf kernel), from
# two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by what the same
# counters read for a plain 256 MiB device copy; see
# profiles/decode_cells512_hbm_traffic.md.  Valid only for the decoder source
# the counters were taken on (at the launch shape named here).
TRAFFIC = {"decoder_sha256_16": "0a361a2a6bff5fcb", "shape": (16, 3, 0, 0), "bytes": 655371445}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def decoder_hash():
    """sha256 prefix of the decoder's sources (kernels and the table format)."""
    h = hashlib.sha256()
    for f in ("csv_decode.hip", "csv_format.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2308_16619_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def record_bytes(blob: bytes, ids, lod: int) -> int:
    """Algorithmic compressed bytes a decode at `lod` must read: record
    header, palette, lane states and the words of the decoded prefix (all
    words for full LOD)."""
    B = int(np.frombuffer(blob, np.uint32, 1, 36)[0])
    idx = np.frombuffer(blob, np.uint64, B + 1, 128)
    sizes = np.diff(idx).astype(np.int64)
    return int(sizes[np.asarray(ids)].sum())


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
    return {"fps": fps, "requests_per_frame": round(len(ids) / nf, 1), "runs": runs}


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
                 "joined": int(st["joined"]), "evictions": int(st["evictions"]), "rebuilds": int(st["rebuilds"]),
                 "batches": int(st["batches"]), "decoded_gb": round(st["decoded_bytes"] / 1e9, 3),
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
    # frames: stage, decode at full LOD, release
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
    med = lambda v: sorted(v)[len(v) // 2]
    staged_bytes = host if done == B else None
    return {"record_bytes": rec, "hbm_record_bytes": rec - host, "host_detail_bytes": host,
            "detail_frac": round(host / rec, 4), "add_volume_s": round(add_s, 3),
            "lod1_ms_split": round(split_ms, 4), "lod1_ms_whole": round(whole_ms, 4),
            "frame": {"bricks": done, "staging_bytes": 8 << 20, "detail_bytes": staged_bytes,
                      "stage_ms": round(med(st), 4), "decode_ms": round(med(dec), 4),
                      "wall_ms": round(med(wall), 4),
                      "stage_gbs": round(staged_bytes / (med(st) * 1e-3) / 1e9, 2) if staged_bytes else None},
            "unstaged_full_lod_ms": round(fb_ms, 4)}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--plain-bricks", type=int, default=1024, help="bricks in the per-brick-launch baseline")
    ap.add_argument("--serving", choices=["full", "none"], default="full",
                    help="serving leg: the 2048x2048x1024 neurite pool with camera-path traces (full) or none")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="measured trace length per serving run")
    ap.add_argument("--detail", choices=["full", "none"], default="full",
                    help="detail-separation leg (a second pool of the volume with level-0 detail in host memory)")
    ap.add_argument("--encoder", choices=["full", "none"], default="full",
                    help="GPU compressor leg (the same volume compressed on the device)")
    ap.add_argument("--shape", default="", help="fixed launch shape 'waves,groups,queue,lpt' instead of the autotuner")
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

    log("generating 512^3 cells volume")
    t0 = time.time()
    vol = synth.cells(n=512, grid=37, p_noise=0.5, seed=2)
    log("generated in %.1fs; encoding" % (time.time() - t0))
    host_threads = 16
    t0 = time.perf_counter()
    blob = csv.encode_volume(vol, threads=host_threads)
    host_s = time.perf_counter() - t0
    info = csv.blob_info(blob)
    log("encoded in %.1fs: %d bytes, CR %.3f%%" % (host_s, len(blob), 100.0 * len(blob) / vol.nbytes))

    pool = csv.Pool(0)
    pool.add_volume(blob)
    B = info["n_bricks"]
    lod = 0
    ids_np = np.arange(B, dtype=np.uint32)
    ids = torch.from_numpy(ids_np.view(np.int32)).to(dev)
    elems = B * 32 ** 3
    out = torch.empty(elems, dtype=torch.int32, device=dev)
    out_bytes = elems * 4
    in_bytes = record_bytes(blob, ids_np, lod)

    stream = torch.cuda.current_stream()
    if args.shape:
        # a fixed launch shape (profiling runs that must compare like with like)
        shape = tuple(int(v) for v in args.shape.split(","))
        pool.set_shape(shape)
        log("fixed shape %s" % (shape,))
    else:
        # the launch shape is picked on this request set by the autotuner
        shape, tune_ms = pool.autotune(ids, out, lod=lod, reps=3)
        torch.cuda.synchronize()
        assert pool.last_error()[0] == 0
        log("autotuned shape %s: %.4f ms" % (shape, tune_ms))
    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        pool.decode(ids, out, lod=lod)
    torch.cuda.synchronize()
    code, who = pool.last_error()
    assert code == 0, ("decode error", code, who)
    # spot check against the input volume (full LOD is lossless)
    got = out.view(B, 32, 32, 32)
    for bid in (0, 1234, B - 1):
        bx, by, bz = bid % 16, (bid // 16) % 16, bid // 256
        ref = torch.from_numpy(vol[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32].astype(np.int64))
        assert torch.equal(got[bid].cpu().to(torch.int64) & 0xFFFFFFFF, ref), bid

    log("timing %d steps" % args.steps)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        pool.decode(ids, out, lod=lod)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1) / args.steps
    gbs = out_bytes / (ms * 1e-3) / 1e9
    code, who = pool.last_error()
    assert code == 0, ("decode error", code, who)


    # per-call time: one decode call (front + leaf kernel) per step, so the event time per step
    achieved = (in_bytes + out_bytes) / (ms * 1e-3) / 1e9
    src_hash = decoder_hash()
    # counters taken on this decoder source (at the launch shape TRAFFIC names), else none
    traffic = TRAFFIC["bytes"] if src_hash == TRAFFIC["decoder_sha256_16"] else None

    # empty-space test (Sec. 4) of the same requests under a transfer
    # function that shows a seeded 1 in 200 of the labels (a brick holds
    # about 100, so the test splits the bricks)
    n_lab = int(vol.max()) + 1
    show = np.random.default_rng(11).random(n_lab) < 0.005
    words = np.zeros((n_lab + 31) // 32, np.uint32)
    nzl = np.nonzero(show)[0].astype(np.uint64)
    np.bitwise_or.at(words, (nzl >> 5).astype(np.int64), (np.uint64(1) << (nzl & np.uint64(31))).astype(np.uint32))
    d_words = torch.from_numpy(words.view(np.int32)).to(dev)
    vmask = torch.empty(B, dtype=torch.uint8, device=dev)
    for _ in range(3):
        pool.visible(ids, d_words, n_lab, out=vmask)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(20):
        pool.visible(ids, d_words, n_lab, out=vmask)
    ev1.record(stream)
    torch.cuda.synchronize()
    vis_us = ev0.elapsed_time(ev1) / 20 * 1e3
    assert pool.last_error()[0] == 0
    visibility = {"bricks": B, "us_per_call": round(vis_us, 2), "bricks_per_s": round(B / (vis_us * 1e-6), 1),
                  "visible_frac": round(float(vmask.float().mean().item()), 4),
                  "transfer_function": "a seeded 1 in 200 of the %d labels visible" % n_lab}

    # baseline: one launch per brick
    nb = min(args.plain_bricks, B)
    pids = ids[:nb].contiguous()
    pout = out[:nb * 32 ** 3]
    pool.decode(pids, pout, lod=lod, plain=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    pool.decode(pids, pout, lod=lod, plain=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1)
    plain_gbs = nb * 32 ** 3 * 4 / (plain_ms * 1e-3) / 1e9
    assert pool.last_error()[0] == 0

    detail = None
    if args.detail == "full":
        log("detail separation leg")
        detail = detail_leg(csv, torch, blob, ids_np, ids, out, shape, pool)

    encoder = None
    if args.encoder == "full":
        log("GPU compressor leg")
        encoder = encoder_leg(csv, torch, vol, blob, host_s, host_threads)

    cpu = None
    if not args.no_cpu:
        import oracle
        oracle._load()
        log("CPU oracle baseline (~%.0fs)" % args.cpu_seconds)
        reps, t0 = 0, time.perf_counter()
        lods = np.zeros(B, np.uint8)
        while True:
            oracle.decode_bricks(blob, ids_np, lods)
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or reps >= 200:
                break
        cpu = {"value": round(reps * out_bytes / el / 1e9, 4), "unit": "GB/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "%d full passes over the same 4096 bricks at full LOD (%.1f s)" % (reps, el)}

    serving = None
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
        "config": {"workload": "512^3 uint32 cells volume (50,653 labels, jittered-grid Voronoi with 1-voxel "
                               "boundary noise), 4096 bricks of 32^3 decoded at full LOD in one launch",
                   "bricks": B, "lod": lod, "compressed_bytes": len(blob),
                   "compression_ratio_pct": round(100.0 * len(blob) / vol.nbytes, 4)},
        "voxels_per_s": round(elems / (ms * 1e-3), 1),
        "wall_s": round(t_wall, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "traffic_shape": list(TRAFFIC["shape"]) if traffic is not None else None,
                     "traffic_unit": "bytes per decode call", "algorithmic_bytes_per_launch": in_bytes + out_bytes,
                     "kernel": "csv_decode_bricks = front_kernel + leaf_kernel", "shape": list(shape),
                     "decoder_sha256_16": src_hash},
        "plain_per_brick_launch": {"value": round(plain_gbs, 3), "unit": "GB/s", "bricks": nb},
        "visibility_test": visibility,
        "detail_separation": detail,
        "encoder": encoder,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
