"""GPU parity of the generic decoder (brick edges 2..64, rANS and raw
nibbles; Table 1's variants) against the oracle, element by element,
through the C ABI."""
import numpy as np
import pytest

import synth
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def log(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module")
def csvlib():
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    return csv


def decode(csv, pool, ids, lods, N, status=False):
    """Requests packed back to back (per-request LODs); returns the output,
    the pool's error word and the per-request status."""
    torch = torch_cuda()
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    lods = np.ascontiguousarray(np.broadcast_to(np.asarray(lods, dtype=np.uint8), ids.shape))
    off, tot = csv.output_offsets(np.minimum(lods, N), brick_log2=N)
    out = torch.full((max(tot, 1),), -1, dtype=torch.int32, device="cuda")
    st = torch.zeros(len(ids), dtype=torch.int32, device="cuda")
    pool.decode(torch.from_numpy(ids.view(np.int32)).cuda(), out, lods=torch.from_numpy(lods).cuda(),
                out_offsets=torch.from_numpy(off.view(np.int64)).cuda(), status=st if status else None)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)[:tot], pool.last_error(), st.cpu().numpy()


def volume(N, seed):
    """A volume of 8 to 64 bricks of edge 2^N mixing Voronoi cells, random
    labels (large palettes), a checkerboard and a uniform region."""
    b = 1 << N
    n = max(32, 4 * b) if N < 6 else 128
    vol = synth.voronoi_bg(n=n, sites=30 + 20 * N, bg=0.2, seed=seed)
    rng = np.random.default_rng(seed)
    vol[:b, :b, :b] = rng.integers(1, 3000, size=(b, b, b)).astype(np.uint32)
    z, y, x = np.meshgrid(np.arange(b), np.arange(b), np.arange(b), indexing="ij")
    if n >= 2 * b:
        vol[:b, :b, b:2 * b] = np.where((x + y + z) % 2 == 0, 7, 9).astype(np.uint32)
        vol[b:2 * b, :b, :b] = 5
        vol[:b, b:2 * b, :b] = rng.integers(1, 18, size=(b, b, b)).astype(np.uint32)  # many P_delta
    return vol


@pytest.mark.parametrize("coding", ["rans", "raw"])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_every_brick_every_lod(csvlib, orc, N, coding):
    vol = volume(N, 30 + N)
    blob = orc.encode_volume(vol, brick_log2=N, scale_bits=10, lane_k=64, tables=0 if coding == "raw" else 2)
    pool = csvlib.Pool()
    assert pool.add_volume(blob) == 0
    assert pool.info()["brick_log2"] == N
    B = orc.volume_info(blob)["n_bricks"]
    ids = np.arange(B)
    for t in range(N + 1):
        log("generic b=%d %s lod %d (%d bricks)" % (1 << N, coding, t, B))
        got, err, _ = decode(csvlib, pool, ids, t, N)
        assert err == (0, 0)
        np.testing.assert_array_equal(got, orc.decode_bricks(blob, ids, [t] * B))
    # full LOD is lossless
    b = 1 << N
    got, _, _ = decode(csvlib, pool, [0], 0, N)
    np.testing.assert_array_equal(got.reshape(b, b, b), vol[:b, :b, :b])


@pytest.mark.parametrize("N", [4, 6])
def test_mixed_lods_codings_and_packed_output(csvlib, orc, N):
    # one pool with a rANS and a raw volume of the same brick size; mixed
    # per-request levels with repeats; then all at one level packed back to
    # back (no offsets)
    torch = torch_cuda()
    v1, v2 = volume(N, 50 + N), volume(N, 60 + N)
    b1 = orc.encode_volume(v1, brick_log2=N, scale_bits=11, lane_k=16)
    b2 = orc.encode_volume(v2, brick_log2=N, tables=0)
    pool = csvlib.Pool()
    pool.add_volume(b1)
    n1 = orc.volume_info(b1)["n_bricks"]
    assert pool.add_volume(b2) == n1
    n2 = orc.volume_info(b2)["n_bricks"]
    rng = np.random.default_rng(N)
    ids = rng.integers(0, n1 + n2, 300)
    lods = rng.integers(0, N + 1, 300)
    log("generic b=%d mixed" % (1 << N))
    got, err, _ = decode(csvlib, pool, ids, lods, N)
    assert err == (0, 0)
    want = [orc.decode_brick(b1, int(i), int(t)) if i < n1 else orc.decode_brick(b2, int(i) - n1, int(t))
            for i, t in zip(ids, lods)]
    np.testing.assert_array_equal(got, np.concatenate([w.ravel() for w in want]))
    g = (1 << N) >> 1
    d_ids = torch.from_numpy(ids.astype(np.uint32).view(np.int32)).cuda()
    out = torch.full((len(ids) * g ** 3,), -1, dtype=torch.int32, device="cuda")
    pool.decode(d_ids, out, lod=1)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    want = [orc.decode_brick(b1, int(i), 1) if i < n1 else orc.decode_brick(b2, int(i) - n1, 1) for i in ids]
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), np.concatenate([w.ravel() for w in want]))
    # one launch per brick gives the same
    log("generic b=%d per-brick launches" % (1 << N))
    k = 20
    off, tot = csvlib.output_offsets(lods[:k].astype(np.uint8), brick_log2=N)
    out = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    pool.decode(torch.from_numpy(ids[:k].astype(np.uint32).view(np.int32)).cuda(), out,
                lods=torch.from_numpy(lods[:k].astype(np.uint8)).cuda(),
                out_offsets=torch.from_numpy(off.view(np.int64)).cuda(), plain=True)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    want = [orc.decode_brick(b1, int(i), int(t)) if i < n1 else orc.decode_brick(b2, int(i) - n1, int(t))
            for i, t in zip(ids[:k], lods[:k])]
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), np.concatenate([w.ravel() for w in want]))


def test_raw_32_cube_pool_and_plain_launches(csvlib, orc):
    vol = synth.cells(n=64, grid=7, seed=12)
    blob = orc.encode_volume(vol, tables=0)
    pool = csvlib.Pool()
    pool.add_volume(blob)
    torch = torch_cuda()
    ids = np.array([3, 0, 7, 7, 1], np.uint32)
    lods = np.array([0, 2, 1, 0, 5], np.uint8)
    off, tot = csvlib.output_offsets(lods)
    out = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    log("raw 32^3, plain launches")
    pool.decode(torch.from_numpy(ids.view(np.int32)).cuda(), out, lods=torch.from_numpy(lods).cuda(),
                out_offsets=torch.from_numpy(off.view(np.int64)).cuda(), plain=True)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), orc.decode_bricks(blob, ids, lods))


def test_errors_are_reported_per_request(csvlib, orc):
    N = 4
    vol = volume(N, 70)
    blob = orc.encode_volume(vol, brick_log2=N, tables=0)
    info = orc.volume_info(blob)
    B = info["n_bricks"]
    idx = np.frombuffer(blob, np.uint64, B + 1, 128)
    rs = (128 + 8 * (B + 1) + 15) & ~15
    # a brick whose first segment is the root's 8 operations alone (no
    # delta), so that its first nibble is an operation: set to code 7
    hit = None
    for bid in range(2, B):
        w = np.frombuffer(blob, np.uint32, 3 + N, rs + int(idx[bid]))
        if int(w[0]) >= 2 and int(w[3 + N - 1]) == 8:
            hit = bid
            break
    assert hit is not None
    P = int(np.frombuffer(blob, np.uint32, 1, rs + int(idx[hit]))[0])
    bad = bytearray(blob)
    bad[rs + int(idx[hit]) + 4 * (3 + N + P)] |= 0x07
    pool = csvlib.Pool()
    pool.add_volume(bytes(bad))
    ids = np.array([1, hit, 10 ** 6, 3, 0], np.uint32)
    lods = np.array([0, 0, 0, 9, 1], np.uint8)
    log("generic errors")
    got, err, st = decode(csvlib, pool, ids, lods, N, status=True)
    assert err[0] != 0
    assert list(st) == [0, csvlib.CSV_ECORRUPT, csvlib.CSV_ERANGE, csvlib.CSV_ERANGE, 0]
    off, _ = csvlib.output_offsets(np.minimum(lods, N), brick_log2=N)
    np.testing.assert_array_equal(got[:4096], orc.decode_brick(blob, 1, 0).ravel())
    np.testing.assert_array_equal(got[4096:8192], 0)
    np.testing.assert_array_equal(got[int(off[4]):int(off[4]) + 512], orc.decode_brick(blob, 0, 1).ravel())


def test_paths_for_32_cube_rans_only_refuse_other_pools(csvlib, orc):
    torch = torch_cuda()
    v16 = orc.encode_volume(volume(4, 80), brick_log2=4)
    v32 = orc.encode_volume(synth.voronoi_bg(n=64, sites=50, seed=3))
    p32 = csvlib.Pool()
    p32.add_volume(v32)
    with pytest.raises(csvlib.CsvError) as e:  # one brick size per pool
        p32.add_volume(v16)
    assert e.value.code == csvlib.CSV_EINVAL
    p16 = csvlib.Pool()
    p16.add_volume(v16)
    ids = torch.zeros(4, dtype=torch.int32, device="cuda")
    out = torch.empty(4 * 4096, dtype=torch.int32, device="cuda")
    for call in (lambda: p16.decode_noalloc(ids, out), lambda: p16.graph(ids, out),
                 lambda: csvlib.Server(p16, cache_bytes=1 << 24), lambda: csvlib.FrameCache(p16, 1 << 24, 16)):
        with pytest.raises(csvlib.CsvError) as e:
            call()
        assert e.value.code == csvlib.CSV_EINVAL
    with pytest.raises(csvlib.CsvError):
        csvlib.Pool().add_volume(v16, detail_host=True)
