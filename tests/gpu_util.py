"""Helpers for the GPU parity tests: run the HIP decoder through the C ABI."""
import numpy as np


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def gpu_decode(pool, ids, lods, plain=False, check_error=True):
    """Decode requests (global ids, per-request LODs) packed back to back;
    returns a numpy uint32 array and the pool's error word."""
    import paper_2308_16619_amd as csv
    torch = torch_cuda()
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    lods = np.ascontiguousarray(np.broadcast_to(np.asarray(lods, dtype=np.uint8), ids.shape))
    off, tot = csv.output_offsets(lods)
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_lods = torch.from_numpy(lods).cuda()
    d_off = torch.from_numpy(off.view(np.int64)).cuda()
    out = torch.full((max(tot, 1),), -1, dtype=torch.int32, device="cuda")
    pool.decode(d_ids, out, lods=d_lods, out_offsets=d_off, plain=plain)
    torch.cuda.synchronize()
    err = pool.last_error()
    if check_error:
        assert err[0] == 0, err
    return out.cpu().numpy().view(np.uint32)[:tot], err


def gpu_decode_uniform(pool, ids, lod):
    """All requests at one LOD, output slot i at i * (32 >> lod)^3."""
    torch = torch_cuda()
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    g = 32 >> lod
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    out = torch.full((len(ids) * g ** 3,), -1, dtype=torch.int32, device="cuda")
    pool.decode(d_ids, out, lod=lod)
    torch.cuda.synchronize()
    assert pool.last_error()[0] == 0
    return out.cpu().numpy().view(np.uint32)
