"""Format sweep: compression ratio, compression time and GPU decode
throughput across the encoder's format parameters (Table 1's study, on a
seeded synthetic volume):

* brick edge 2^brick_log2 in {16, 32, 64}, each with Table 1's three
  entropy-coding variants: no rANS (the symbol stream stored as raw
  nibbles, csv_encode_opts.coding 1), rANS with one frequency table for all
  symbols, rANS with two (levels >= 1 and L_0: the default).  32^3 rANS
  bricks decode with the tuned kernels, the others with the generic
  decoder;
* interleaved rANS states per brick W (lane_max) in {1, 4, 16, 64} (W = 1 is
  the paper's single stream per brick);
* table precision scale_bits in {8, 9, 10, 11}.

Each variant prints one JSON line: compressed bytes and ratio, host
compression seconds (16 threads), the decode of every brick at full LOD in
one call (HIP events over `reps` calls, the tuned shape for 32^3 rANS;
output checked against the volume), and for 32^3 rANS bricks the GPU
compressor's time.

    python -m paper_2308_16619_amd.format_sweep [--n 512] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def decode_rate(csv, torch, vol, blob, reps, log2=5):
    """GB/s of uint32 labels for all bricks of blob at full LOD."""
    b = 1 << log2
    nz, ny, nx = vol.shape
    nb = (nx // b) * (ny // b) * (nz // b)
    pool = csv.Pool(0)
    pool.add_volume(blob)
    ids = torch.arange(nb, dtype=torch.int32, device="cuda")
    out = torch.empty(nb * b ** 3, dtype=torch.int32, device="cuda")
    shape = None
    if log2 == 5 and csv.blob_info(blob)["coding"] == 0:
        shape, _ = pool.autotune(ids, out, lod=0, reps=2)
        shape = list(shape)
    pool.decode(ids, out, lod=0)
    torch.cuda.synchronize()
    assert pool.last_error()[0] == 0
    # lossless: full LOD is the volume, brick by brick
    ref = torch.from_numpy(vol.view(np.int32)).cuda()
    ref = ref.view(nz // b, b, ny // b, b, nx // b, b).permute(0, 2, 4, 1, 3, 5).reshape(-1)
    assert torch.equal(out, ref), "decode differs from the volume"
    del ref
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pool.decode(ids, out, lod=0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return out.numel() * 4 / (ms * 1e-3) / 1e9, ms, shape


def host_encode(csv, vol, **kw):
    t0 = time.perf_counter()
    blob = csv.encode_volume(vol, threads=16, **kw)
    return blob, time.perf_counter() - t0


def gpu_encode_ms(csv, torch, vol, blob, **kw):
    d = torch.from_numpy(vol.view(np.int32)).cuda()
    assert csv.encode_volume_gpu(d, **kw) == blob, "GPU container differs"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    csv.encode_volume_gpu(d, **kw)
    return (time.perf_counter() - t0) * 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512, help="edge of the cells volume")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-gpu", action="store_true", help="compression ratios only")
    args = ap.parse_args()
    import synth
    import paper_2308_16619_amd as csv
    torch = None
    if not args.no_gpu:
        import torch
    vol = synth.cells(n=args.n, grid=max(2, round(37 * args.n / 512)), seed=2)
    raw = vol.nbytes
    name = "%d^3 cells" % args.n
    # Table 1: brick edge x entropy coding
    for log2 in (4, 5, 6):
        for tables, coding in ((2, 0), (1, 0), (2, 1)):
            blob, sec = host_encode(csv, vol, brick_log2=log2, tables=tables, coding=coding)
            label = "no rANS (raw nibbles)" if coding else "rANS, %d table%s" % (tables, "s" * (tables > 1))
            rec = {"volume": name, "brick": 1 << log2, "coding": label, "scale_bits": 10, "lane_max": 64,
                   "compressed_bytes": len(blob), "compression_ratio_pct": round(100.0 * len(blob) / raw, 4),
                   "host_encode_s": round(sec, 3), "host_encode_gbs": round(raw / sec / 1e9, 3)}
            if torch is not None:
                if log2 == 5 and coding == 0:
                    rec["gpu_encode_ms"] = round(gpu_encode_ms(csv, torch, vol, blob, tables=tables), 3)
                gbs, ms, shape = decode_rate(csv, torch, vol, blob, args.reps, log2)
                rec.update({"decode_gbs": round(gbs, 2), "ms_per_call": round(ms, 4),
                            "decoder": "tuned 32^3 kernels" if shape else "generic", "shape": shape})
            print(json.dumps(rec), flush=True)
    # interleaving width and table precision (32^3 bricks, two tables)
    for sbits, lanes in [(10, w) for w in (1, 4, 16)] + [(s, 64) for s in (8, 9, 11)]:
        blob, sec = host_encode(csv, vol, scale_bits=sbits, lane_max=lanes)
        rec = {"volume": name, "brick": 32, "coding": "rANS, 2 tables", "scale_bits": sbits, "lane_max": lanes,
               "compressed_bytes": len(blob), "compression_ratio_pct": round(100.0 * len(blob) / raw, 4),
               "host_encode_s": round(sec, 3)}
        if torch is not None:
            gbs, ms, shape = decode_rate(csv, torch, vol, blob, args.reps)
            rec.update({"decode_gbs": round(gbs, 2), "ms_per_call": round(ms, 4), "shape": shape})
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
