"""GPU parity of the GPU compressor: its container must equal the oracle's
encoder output byte for byte (header, tables, index, every record)."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def log(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def csvlib():
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    return csv


def first_difference(a: bytes, b: bytes):
    n = min(len(a), len(b))
    x = np.frombuffer(a[:n], np.uint8) != np.frombuffer(b[:n], np.uint8)
    return int(np.argmax(x)) if x.any() else n


def check(csvlib, orc, name, vol, **kw):
    opts = {"scale_bits": 10, "lane_k": 64, "lane_max": 64, **kw}
    log("encode %s %s %s" % (name, vol.shape, opts))
    got = csvlib.encode_volume_gpu(vol, **opts)
    want = orc.encode_volume(vol, **opts)
    assert len(got) == len(want) and got == want, \
        "%s: %d vs %d bytes, first difference at byte %d" % (name, len(got), len(want), first_difference(got, want))
    return got


def edge_bricks():
    from test_gpu_decode import golden_volume
    return golden_volume()


@pytest.mark.parametrize("case", ["cfg1", "edge", "padded", "bits8_stride3", "k1_w16", "w1", "bits12_k256",
                                  "one_table"])
def test_gpu_encoder_matches_oracle(csvlib, orc, case):
    if case == "cfg1":
        check(csvlib, orc, case, synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1))
    elif case == "edge":
        # uniform, half, checkerboard, > 32768 distinct labels, long word
        # stream, many P_delta, smooth, zero
        check(csvlib, orc, case, edge_bricks(), scale_bits=11)
    elif case == "padded":
        check(csvlib, orc, case, np.ascontiguousarray(synth.voronoi_bg(n=64, sites=30, seed=3)[:40, :50, :33]))
    elif case == "bits8_stride3":
        check(csvlib, orc, case, synth.voronoi_bg(n=64, sites=90, seed=4), scale_bits=8, sample_stride=3)
    elif case == "k1_w16":
        check(csvlib, orc, case, synth.voronoi_bg(n=64, sites=90, seed=5), lane_k=1, lane_max=16)
    elif case == "w1":
        check(csvlib, orc, case, synth.voronoi_bg(n=64, sites=90, seed=6), lane_max=1)
    elif case == "bits12_k256":
        check(csvlib, orc, case, synth.cells(n=128, grid=9, seed=8), scale_bits=12, lane_k=256)
    else:
        check(csvlib, orc, case, edge_bricks(), tables=1)


def test_one_table_container_decodes(csvlib, orc):
    # Table 1's one-table variant: both header tables equal; the decoder
    # reads it unchanged, at every LOD
    from gpu_util import gpu_decode_uniform
    vol = synth.cells(n=128, grid=9, seed=8)
    blob = check(csvlib, orc, "one_table_cells", vol, tables=1)
    pool = csvlib.Pool()
    pool.add_volume(blob)
    for t in range(6):
        log("one-table container, lod %d" % t)
        np.testing.assert_array_equal(gpu_decode_uniform(pool, np.arange(64), t),
                                      orc.decode_bricks(blob, np.arange(64), [t] * 64))


def test_gpu_encoder_cells_and_round_trip(csvlib, orc):
    torch = torch_cuda()
    vol = synth.cells(n=512, grid=37, seed=2)[:256, :256, :256].copy()
    blob = check(csvlib, orc, "cells256", vol)
    # the pool decodes it back to the volume (full LOD is lossless)
    pool = csvlib.Pool()
    pool.add_volume(blob)
    ids = torch.arange(512, dtype=torch.int32, device="cuda")
    out = torch.empty(512 * 32 ** 3, dtype=torch.int32, device="cuda")
    pool.decode(ids, out, lod=0)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    ref = torch.from_numpy(vol.view(np.int32)).cuda()
    ref = ref.view(8, 32, 8, 32, 8, 32).permute(0, 2, 4, 1, 3, 5).reshape(-1)
    assert torch.equal(out, ref)


def test_gpu_encoder_records_beyond_first_arena(csvlib, orc):
    # random labels: records larger than the bricks' raw bytes, more than
    # the first arena holds (the second pass sizes it exactly)
    rng = np.random.default_rng(17)
    vol = rng.integers(1, 1 << 22, size=(256, 128, 192)).astype(np.uint32)
    blob = check(csvlib, orc, "random", vol)
    assert len(blob) > 16 << 20


def test_gpu_encoder_input_forms_and_errors(csvlib, orc):
    torch = torch_cuda()
    vol = synth.voronoi_bg(n=64, sites=50, seed=9)
    want = orc.encode_volume(vol, scale_bits=10, lane_k=64)
    d = torch.from_numpy(vol.view(np.int32)).cuda()
    assert csvlib.encode_volume_gpu(d) == want
    torch.cuda.synchronize()
    assert csvlib.encode_volume_gpu(d, stream=torch.cuda.Stream()) == want
    # the kept buffers released, then grown again
    csvlib.encode_gpu_release(0)
    assert csvlib.encode_volume_gpu(vol) == want
    one = np.full((1, 1, 1), 7, np.uint32)
    assert csvlib.encode_volume_gpu(one) == orc.encode_volume(one, scale_bits=10, lane_k=64)
    with pytest.raises(csvlib.CsvError):
        csvlib.encode_volume_gpu(d, brick_log2=4)
    with pytest.raises(csvlib.CsvError):
        csvlib.encode_volume_gpu(d, lane_max=48)


def test_gpu_encoder_full_size_workload(csvlib, orc):
    # the benchmark's 512^3 cells volume (4096 bricks), in the launch
    # configuration the benchmark times, against the oracle's container
    vol = synth.cells(n=512, grid=37, p_noise=0.5, seed=2)
    blob = check(csvlib, orc, "cells512", vol)
    assert csvlib.blob_info(blob)["n_bricks"] == 4096
