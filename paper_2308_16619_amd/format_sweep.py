"""Format sweep: compression ratio and GPU decode throughput across the
encoder's format parameters (Table 1's study, on a seeded synthetic volume):

* brick edge 2^brick_log2 in {16, 32, 64} (the GPU decoder takes 32^3
  bricks, so the other edges report the compression ratio only);
* interleaved rANS states per brick W (lane_max) in {1, 4, 16, 64} (W = 1 is
  the paper's single stream per brick);
* table precision scale_bits in {8, 9, 10, 11}.

Each variant prints one JSON line: compressed bytes and ratio, and for 32^3
bricks the decode of every brick at full LOD in one call (autotuned launch
shape, HIP events over `reps` calls; output checked against the volume).

    python -m paper_2308_16619_amd.format_sweep [--n 512] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def decode_rate(csv, torch, vol, blob, reps):
    """GB/s of uint32 labels for all bricks of blob at full LOD (32^3 bricks)."""
    nz, ny, nx = vol.shape
    nb = (nx // 32) * (ny // 32) * (nz // 32)
    pool = csv.Pool(0)
    pool.add_volume(blob)
    ids = torch.arange(nb, dtype=torch.int32, device="cuda")
    out = torch.empty(nb * 32 ** 3, dtype=torch.int32, device="cuda")
    shape, _ = pool.autotune(ids, out, lod=0, reps=2)
    pool.decode(ids, out, lod=0)
    torch.cuda.synchronize()
    assert pool.last_error()[0] == 0
    # lossless: full LOD is the volume, brick by brick
    ref = torch.from_numpy(vol.view(np.int32)).cuda()
    ref = ref.view(nz // 32, 32, ny // 32, 32, nx // 32, 32).permute(0, 2, 4, 1, 3, 5).reshape(-1)
    assert torch.equal(out, ref), "decode differs from the volume"
    del ref
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pool.decode(ids, out, lod=0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return out.numel() * 4 / (ms * 1e-3) / 1e9, ms, list(shape)


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
    variants = [(b, 10, 64) for b in (4, 5, 6)] + [(5, 10, w) for w in (1, 4, 16)] + \
               [(5, s, 64) for s in (8, 9, 11)]
    for log2, sbits, lanes in variants:
        blob = csv.encode_volume(vol, brick_log2=log2, scale_bits=sbits, lane_max=lanes)
        rec = {"volume": "%d^3 cells" % args.n, "brick": 1 << log2, "scale_bits": sbits, "lane_max": lanes,
               "compressed_bytes": len(blob), "compression_ratio_pct": round(100.0 * len(blob) / raw, 4)}
        if log2 == 5 and torch is not None:
            gbs, ms, shape = decode_rate(csv, torch, vol, blob, args.reps)
            rec.update({"decode_gbs": round(gbs, 2), "ms_per_call": round(ms, 4), "shape": shape})
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
