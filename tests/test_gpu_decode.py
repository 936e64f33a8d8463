"""GPU parity: the HIP decoder against the oracle, element by element."""
import os
import sys

import numpy as np
import pytest

import synth
from gpu_util import gpu_decode, gpu_decode_uniform, torch_cuda

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def log(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def csvlib():
    torch_cuda()
    import paper_2308_16619_amd as csv
    csv.lib()
    return csv


@pytest.fixture(scope="module")
def cfg1(orc):
    vol = synth.voronoi_bg(n=64, sites=200, bg=0.30, seed=1)
    return vol, orc.encode_volume(vol, scale_bits=10, lane_k=64)


def test_config1_every_brick_every_lod(csvlib, orc, cfg1):
    vol, blob = cfg1
    pool = csvlib.Pool()
    first = pool.add_volume(blob)
    assert first == 0
    for t in range(6):
        log("cfg1 lod %d" % t)
        got = gpu_decode_uniform(pool, np.arange(8), t)
        want = orc.decode_bricks(blob, np.arange(8), [t] * 8)
        np.testing.assert_array_equal(got, want)


def test_config1_mixed_lods_and_repeats(csvlib, orc, cfg1):
    vol, blob = cfg1
    pool = csvlib.Pool()
    pool.add_volume(blob)
    rng = np.random.default_rng(3)
    ids = rng.integers(0, 8, 300)
    lods = rng.integers(0, 6, 300)
    log("cfg1 mixed")
    got, _ = gpu_decode(pool, ids, lods)
    np.testing.assert_array_equal(got, orc.decode_bricks(blob, ids, lods))


def golden_volume():
    z, y, x = np.meshgrid(np.arange(32), np.arange(32), np.arange(32), indexing="ij")
    A, B = 17, 4
    uniform = np.full((32, 32, 32), A, np.uint32)
    half = np.where(x < 16, A, B).astype(np.uint32)
    checker = np.where((x + y + z) % 2 == 0, A, B).astype(np.uint32)
    rng = np.random.default_rng(12)
    distinct = rng.permutation(1 << 20)[:32768].astype(np.uint32).reshape(32, 32, 32) + 1  # P > 32768
    many = rng.integers(1, 6000, size=(32, 32, 32)).astype(np.uint32)  # P > 4096, long word stream
    delta_heavy = rng.integers(1, 18, size=(32, 32, 32)).astype(np.uint32)  # many P_delta
    smooth = synth.random_brick(32, 9, 5, smooth=8)
    bricks = [uniform, half, checker, distinct, many, delta_heavy, smooth, np.zeros((32, 32, 32), np.uint32)]
    return np.concatenate(bricks, axis=2)


def test_edge_bricks(csvlib, orc):
    vol = golden_volume()
    blob = orc.encode_volume(vol, scale_bits=11, lane_k=64)
    pool = csvlib.Pool()
    pool.add_volume(blob)
    n = vol.shape[2] // 32
    for t in range(6):
        log("edge bricks lod %d" % t)
        got = gpu_decode_uniform(pool, np.arange(n), t)
        np.testing.assert_array_equal(got, orc.decode_bricks(blob, np.arange(n), [t] * n))
    # full LOD is lossless
    got = gpu_decode_uniform(pool, np.arange(n), 0).reshape(n, 32, 32, 32)
    for i in range(n):
        np.testing.assert_array_equal(got[i], vol[:, :, 32 * i:32 * (i + 1)])


@pytest.mark.parametrize("scale_bits,lane_k,lane_max", [(8, 1, 64), (11, 1000000, 64), (10, 16, 8), (11, 64, 1),
                                                        (12, 64, 64), (12, 256, 16)])
def test_format_parameters(csvlib, orc, scale_bits, lane_k, lane_max):
    vol = synth.voronoi_bg(n=64, sites=300, bg=0.2, seed=scale_bits + lane_k)
    blob = orc.encode_volume(vol, scale_bits=scale_bits, lane_k=lane_k, lane_max=lane_max)
    pool = csvlib.Pool()
    pool.add_volume(blob)
    for t in (0, 1, 3):
        log("format S=%d K=%d Wmax=%d lod %d" % (scale_bits, lane_k, lane_max, t))
        got = gpu_decode_uniform(pool, np.arange(8), t)
        np.testing.assert_array_equal(got, orc.decode_bricks(blob, np.arange(8), [t] * 8))


def test_twelve_bit_tables_in_lds_and_in_global_memory(csvlib, orc, cfg1):
    # one 12-bit volume: its two tables (32 KiB) are copied to LDS; with a
    # 10-bit volume beside it the tables no longer fit and are read from
    # global memory.  Both decode to the oracle's bytes.
    vol, blob = cfg1
    v12 = synth.cells(n=128, grid=9, seed=8)
    b12 = orc.encode_volume(v12, scale_bits=12, lane_k=64)
    solo = csvlib.Pool()
    solo.add_volume(b12)
    log("12-bit tables, LDS")
    for t in (0, 1):
        got = gpu_decode_uniform(solo, np.arange(64), t)
        np.testing.assert_array_equal(got, orc.decode_bricks(b12, np.arange(64), [t] * 64))
    both = csvlib.Pool()
    assert both.add_volume(b12) == 0 and both.add_volume(blob) == 64
    rng = np.random.default_rng(12)
    ids = rng.integers(0, 72, 400)
    lods = rng.integers(0, 4, 400)
    log("12-bit and 10-bit tables, global memory")
    got, _ = gpu_decode(both, ids, lods)
    want = [orc.decode_brick(b12, int(i), int(t)) if i < 64 else orc.decode_brick(blob, int(i) - 64, int(t))
            for i, t in zip(ids, lods)]
    np.testing.assert_array_equal(got, np.concatenate([w.ravel() for w in want]))


@pytest.mark.parametrize("shape", [None, (2, 3, 0, 0, 1)])
def test_plain_per_brick_launch_matches(csvlib, orc, cfg1, shape):
    vol, blob = cfg1
    pool = csvlib.Pool()
    pool.add_volume(blob)
    if shape:
        pool.set_shape(shape)
    ids = np.array([7, 0, 3, 3, 5])
    lods = np.array([0, 1, 2, 0, 4])
    log("plain per-brick launches")
    got, _ = gpu_decode(pool, ids, lods, plain=True)
    np.testing.assert_array_equal(got, orc.decode_bricks(blob, ids, lods))


def test_two_volumes_one_pool(csvlib, orc, cfg1):
    vol, blob = cfg1
    vol2 = synth.blobs(n=128, sites=12, amp=10, seed=4)
    blob2 = orc.encode_volume(vol2, scale_bits=10, lane_k=32)
    pool = csvlib.Pool()
    assert pool.add_volume(blob) == 0
    assert pool.add_volume(blob2) == 8
    rng = np.random.default_rng(8)
    ids = rng.integers(0, 8 + 64, 200)
    lods = rng.integers(0, 3, 200)
    log("two volumes")
    got, _ = gpu_decode(pool, ids, lods)
    want = []
    for i, t in zip(ids, lods):
        want.append(orc.decode_brick(blob, int(i), int(t)) if i < 8 else orc.decode_brick(blob2, int(i) - 8, int(t)))
    np.testing.assert_array_equal(got, np.concatenate([w.ravel() for w in want]))


def test_out_of_range_request_is_reported(csvlib, orc, cfg1):
    vol, blob = cfg1
    pool = csvlib.Pool()
    pool.add_volume(blob)
    ids = np.array([1, 99, 2])
    log("out of range id")
    got, err = gpu_decode(pool, ids, [0, 0, 0], check_error=False)
    assert err == (csvlib.CSV_ERANGE, 1)
    np.testing.assert_array_equal(got[32768:65536], 0)
    np.testing.assert_array_equal(got[:32768], orc.decode_brick(blob, 1, 0).ravel())
    np.testing.assert_array_equal(got[65536:], orc.decode_brick(blob, 2, 0).ravel())
    assert pool.last_error() == (0, 0)


@pytest.mark.parametrize("shape", [None, (2, 3, 0, 0, 1)])
def test_status_names_each_failed_request(csvlib, orc, cfg1, shape):
    # csv_decode_bricks_status: an unknown id, a bad LOD and a corrupt
    # record each mark their own request; the others stay 0 and decode
    # (also with the paired front kernel)
    torch = torch_cuda()
    vol, blob = cfg1
    info = orc.volume_info(blob)
    B = info["n_bricks"]
    idx = np.frombuffer(blob, np.uint64, B + 1, 128)
    rs = (128 + 8 * (B + 1) + 15) & ~15
    w = np.frombuffer(blob, np.uint32, 8, rs + int(idx[6]))
    bad = bytearray(blob)
    bad[rs + int(idx[6]) + 4 * (8 + int(w[0]) + int(w[1])) + 2 * (int(w[2]) // 2)] ^= 0x10
    pool = csvlib.Pool()
    pool.add_volume(bytes(bad))
    if shape:
        pool.set_shape(shape)
    ids = np.array([2, 77, 6, 3, 1], np.uint32)
    lods = np.array([0, 0, 0, 9, 1], np.uint8)
    off, tot = csvlib.output_offsets(np.minimum(lods, 5))
    status = torch.zeros(5, dtype=torch.int32, device="cuda")
    out = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    log("per-request status")
    pool.decode(torch.from_numpy(ids.view(np.int32)).cuda(), out, lods=torch.from_numpy(lods).cuda(),
                out_offsets=torch.from_numpy(off.view(np.int64)).cuda(), status=status)
    torch.cuda.synchronize()
    assert pool.last_error()[0] != 0
    assert status.cpu().tolist() == [0, csvlib.CSV_ERANGE, csvlib.CSV_ECORRUPT, csvlib.CSV_ERANGE, 0]
    got = out.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got[:32768], orc.decode_brick(blob, 2, 0).ravel())
    np.testing.assert_array_equal(got[int(off[4]):int(off[4]) + 4096], orc.decode_brick(blob, 1, 1).ravel())


@pytest.mark.parametrize("shape", [None, (2, 3, 0, 0, 1)])
def test_corrupt_record_is_reported(csvlib, orc, cfg1, shape):
    vol, blob = cfg1
    info = orc.volume_info(blob)
    B = info["n_bricks"]
    idx = np.frombuffer(blob, np.uint64, B + 1, 128)
    rs = (128 + 8 * (B + 1) + 15) & ~15
    w = np.frombuffer(blob, np.uint32, 8, rs + int(idx[4]))
    P, W, nw = int(w[0]), int(w[1]), int(w[2])
    bad = bytearray(blob)
    bad[rs + int(idx[4]) + 4 * (8 + P + W) + 2 * (nw // 2)] ^= 0x10
    pool = csvlib.Pool()
    pool.add_volume(bytes(bad))
    if shape:
        pool.set_shape(shape)
    log("corrupt record, shape %s" % (shape,))
    got, err = gpu_decode(pool, [3, 4, 5], [0, 0, 0], check_error=False)
    assert err == (csvlib.CSV_ECORRUPT, 4)
    np.testing.assert_array_equal(got[32768:65536], 0)
    np.testing.assert_array_equal(got[:32768], orc.decode_brick(blob, 3, 0).ravel())


@pytest.fixture(scope="module")
def cfg2(orc):
    log("generating config 2 (512^3 cells)")
    vol = synth.cells(n=512, grid=37, seed=2)
    return vol, orc.encode_volume(vol, scale_bits=10, lane_k=64)


def test_config2_full_lod(csvlib, orc, cfg2):
    vol, blob = cfg2
    pool = csvlib.Pool()
    pool.add_volume(blob)
    log("cfg2 full LOD, 4096 bricks")
    got = gpu_decode_uniform(pool, np.arange(4096), 0)
    want = orc.decode_bricks(blob, np.arange(4096), [0] * 4096)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("cap", ["0", "1200", "1600", ""])
def test_reference_list_bound(csvlib, orc, cfg2, cap, monkeypatch):
    # the leaf kernel resolves same-level references from a list before the
    # output, or chases them in the output loop for a brick whose list is
    # longer than the bound: at bound 0 every brick chases, in between the
    # cells bricks (about 1.5k references each) split, unbounded none does
    vol, blob = cfg2
    monkeypatch.setenv("CSV_REF_LIST_CAP", cap)
    pool = csvlib.Pool()
    pool.add_volume(blob)
    ids = np.arange(1, 4096, 2)
    log("cfg2 reference list bound %r" % cap)
    got = gpu_decode_uniform(pool, ids, 0)
    np.testing.assert_array_equal(got, orc.decode_bricks(blob, ids, [0] * len(ids)))


@pytest.mark.parametrize("lod", [1, 2, 3])
def test_config2_lower_lods(csvlib, orc, cfg2, lod):
    vol, blob = cfg2
    pool = csvlib.Pool()
    pool.add_volume(blob)
    log("cfg2 lod %d" % lod)
    got = gpu_decode_uniform(pool, np.arange(4096), lod)
    np.testing.assert_array_equal(got, orc.decode_bricks(blob, np.arange(4096), [lod] * 4096))


@pytest.mark.parametrize("shape", [(4, 1, 1), (8, 3, 0), (16, 4, 1), (16, 8, 1), (4, 2, 0), (2, 3, 0), (2, 2, 1)])
def test_launch_shapes_agree(csvlib, orc, cfg2, shape):
    # every launch shape decodes the same bytes; 8 waves per group leave an
    # LDS arena too small for the densest bricks, which then take the
    # global-memory arena path
    torch = torch_cuda()
    vol, blob = cfg2
    pool = csvlib.Pool()
    pool.add_volume(blob)
    ids = np.arange(0, 4096, 3, dtype=np.uint32)
    log("cfg2 shape %s" % (shape,))
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    out = torch.full((len(ids) * 32768,), -1, dtype=torch.int32, device="cuda")
    pool.decode(d_ids, out, lod=0, shape=shape)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    want = orc.decode_bricks(blob, ids, [0] * len(ids))
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), want)


@pytest.mark.parametrize("shape", [(16, 3, 0, 0, 1), (16, 3, 0, 0, 2), (8, 2, 1, 1, 4), (16, 4, 0, 0, 8),
                                   (8, 3, 0, 1, 4), (16, 3, 0, 1, 1), (2, 3, 0, 0, 2), (2, 3, 0, 1, 4)])
def test_pipelined_chunks_agree(csvlib, orc, cfg1, cfg2, shape):
    # the requests split into chunks that alternate between the caller's
    # stream and the pool's second stream: mixed LODs over two volumes with
    # per-request offsets and statuses (one unknown id late in the batch),
    # then every brick of the cells volume at full LOD packed back to back
    torch = torch_cuda()
    pool = csvlib.Pool()
    pool.add_volume(cfg1[1])
    pool.add_volume(cfg2[1])
    ids, lods = mixed_requests(23, 9000, 8 + 4096)
    ids[8500] = 10 ** 6
    off, tot = csvlib.output_offsets(lods)
    want = np.concatenate([np.zeros((32 >> int(t)) ** 3, np.uint32) if i >= 8 + 4096 else
                           orc.decode_brick(cfg1[1], int(i), int(t)).ravel() if i < 8 else
                           orc.decode_brick(cfg2[1], int(i) - 8, int(t)).ravel() for i, t in zip(ids, lods)])
    out = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    status = torch.zeros(len(ids), dtype=torch.int32, device="cuda")
    log("pipelined mixed %s" % (shape,))
    pool.set_shape(shape)
    pool.decode(torch.from_numpy(ids.view(np.int32)).cuda(), out, lods=torch.from_numpy(lods.copy()).cuda(),
                out_offsets=torch.from_numpy(off.view(np.int64)).cuda(), status=status)
    torch.cuda.synchronize()
    assert pool.last_error() == (csvlib.CSV_ERANGE, 8500)
    st = status.cpu().numpy()
    assert st[8500] == csvlib.CSV_ERANGE and np.count_nonzero(st) == 1
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), want)
    log("pipelined full LOD %s" % (shape,))
    d_ids = torch.arange(8, 8 + 4096, dtype=torch.int32, device="cuda")
    out = torch.full((4096 * 32768,), -1, dtype=torch.int32, device="cuda")
    pool.decode(d_ids, out, lod=0)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32),
                                  orc.decode_bricks(cfg2[1], np.arange(4096), [0] * 4096))


def mixed_requests(seed, n, n_bricks):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_bricks, n).astype(np.uint32), rng.integers(0, 3, n).astype(np.uint8)


def test_longest_first_order_and_autotune(csvlib, orc, cfg1, cfg2):
    # mixed LODs over two volumes: the longest-first order and every tuned
    # shape give the oracle's bytes
    torch = torch_cuda()
    pool = csvlib.Pool()
    pool.add_volume(cfg1[1])
    pool.add_volume(cfg2[1])
    ids, lods = mixed_requests(11, 3000, 8 + 4096)
    off, tot = csvlib.output_offsets(lods)
    want = np.concatenate([orc.decode_brick(cfg1[1], int(i), int(t)).ravel() if i < 8 else
                           orc.decode_brick(cfg2[1], int(i) - 8, int(t)).ravel() for i, t in zip(ids, lods)])
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_lods = torch.from_numpy(lods.copy()).cuda()
    d_off = torch.from_numpy(off.view(np.int64)).cuda()
    out = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    log("lpt order")
    pool.decode(d_ids, out, lods=d_lods, out_offsets=d_off, shape=(8, 4, 1, 1))
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), want)
    log("autotune")
    out.fill_(-1)
    shape, ms = pool.autotune(d_ids, out, lods=d_lods, out_offsets=d_off, reps=2)
    assert pool.get_shape() == shape and ms > 0
    out.fill_(-1)
    pool.decode(d_ids, out, lods=d_lods, out_offsets=d_off)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), want)


def test_tuning_file_round_trip(csvlib, orc, cfg1, cfg2, tmp_path):
    # a tuned class written to a file and read into a fresh pool; that
    # pool's decode of the same class uses it and gives the oracle's bytes;
    # a file from another device adds nothing, a malformed one is refused
    torch = torch_cuda()
    pool = csvlib.Pool()
    pool.add_volume(cfg2[1])
    ids = np.arange(0, 4096, 2, dtype=np.uint32)
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    out = torch.full((len(ids) * 32768,), -1, dtype=torch.int32, device="cuda")
    log("tuning save / load")
    shape, _ = pool.autotune(d_ids, out, lod=0, reps=1)
    path = str(tmp_path / "tuning.txt")
    pool.save_tuning(path)
    lines = open(path).read().splitlines()
    assert lines[0].startswith("csv-tuning 1 ") and len(lines) == 2
    fresh = csvlib.Pool()
    fresh.add_volume(cfg2[1])
    assert fresh.load_tuning(path) == 1
    out.fill_(-1)
    fresh.decode(d_ids, out, lod=0)
    torch.cuda.synchronize()
    assert fresh.last_error() == (0, 0)
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), orc.decode_bricks(cfg2[1], ids, [0] * len(ids)))
    other = str(tmp_path / "other.txt")
    head = lines[0].split()
    open(other, "w").write("csv-tuning 1 some-other-gpu %s\n%s\n" % (head[3], lines[1]))
    assert fresh.load_tuning(other) == 0
    bad = str(tmp_path / "bad.txt")
    open(bad, "w").write(lines[0] + "\n12 7 11 16 3 0 0 4 1.0\n")
    with pytest.raises(csvlib.CsvError) as e:
        fresh.load_tuning(bad)
    assert e.value.code == csvlib.CSV_ECORRUPT


@pytest.mark.parametrize("shape", [(16, 4, 1, 0), (8, 5, 1, 1), (2, 3, 0, 1)])
def test_graph_replays(csvlib, orc, cfg2, shape):
    # a captured decode replayed several times, with eager work and
    # synchronisation in between; every replay must match
    torch = torch_cuda()
    vol, blob = cfg2
    pool = csvlib.Pool()
    pool.add_volume(blob)
    pool.set_shape(shape)
    ids, lods = mixed_requests(5, 1500, 4096)
    off, tot = csvlib.output_offsets(lods)
    want = orc.decode_bricks(blob, ids, lods)
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_lods = torch.from_numpy(lods.copy()).cuda()
    d_off = torch.from_numpy(off.view(np.int64)).cuda()
    out = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    log("graph capture %s" % (shape,))
    g = pool.graph(d_ids, out, lods=d_lods, out_offsets=d_off, stream=s)
    for rep in range(4):
        out.fill_(-1)
        torch.cuda.synchronize()
        g.launch(stream=s)
        s.synchronize()
        assert pool.last_error() == (0, 0)
        np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), want, err_msg="replay %d" % rep)
        pool.decode(d_ids[:7].contiguous(), torch.empty(7 * 32768, dtype=torch.int32, device="cuda"), lod=0)
        torch.cuda.synchronize()
    g.close()


@pytest.mark.parametrize("shape", [(16, 3, 0, 0, 1), (8, 3, 1, 1, 4), (2, 3, 0, 0, 1)])
def test_device_count_decodes_a_prefix(csvlib, orc, cfg1, cfg2, shape):
    # csv_decode_bricks_devcount: the kernels decode min(n_max, *n_dev)
    # requests and leave the other outputs untouched (a lpt or chunked shape
    # runs as one launch pair without the order)
    torch = torch_cuda()
    pool = csvlib.Pool()
    pool.add_volume(cfg1[1])
    pool.add_volume(cfg2[1])
    pool.set_shape(shape)
    n_max = 2500
    ids, lods = mixed_requests(31, n_max, 8 + 4096)
    off, tot = csvlib.output_offsets(lods)
    ref = [orc.decode_brick(cfg1[1], int(i), int(t)).ravel() if i < 8 else
           orc.decode_brick(cfg2[1], int(i) - 8, int(t)).ravel() for i, t in zip(ids, lods)]
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_lods = torch.from_numpy(lods.copy()).cuda()
    d_off = torch.from_numpy(off.view(np.int64)).cuda()
    for k in (0, 1, 1777, n_max, 10 ** 6):
        log("device count %d of %d, shape %s" % (k, n_max, shape))
        out = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
        cnt = torch.tensor([k], dtype=torch.int32, device="cuda")
        pool.decode_devcount(d_ids, out, cnt, lods=d_lods, out_offsets=d_off)
        torch.cuda.synchronize()
        assert pool.last_error() == (0, 0)
        got = out.cpu().numpy().view(np.uint32)
        m = min(k, n_max)
        end = int(off[m]) if m < n_max else tot
        np.testing.assert_array_equal(got[:end], np.concatenate(ref[:m]) if m else got[:0])
        assert (got[end:] == 0xFFFFFFFF).all()
    # packed outputs at one LOD
    g = 32 >> 1
    out = torch.full((300 * g ** 3,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.tensor([123], dtype=torch.int32, device="cuda")
    pool.decode_devcount(d_ids[:300].contiguous(), out, cnt, lod=1)
    torch.cuda.synchronize()
    want = np.concatenate([orc.decode_brick(cfg1[1], int(i), 1).ravel() if i < 8 else
                           orc.decode_brick(cfg2[1], int(i) - 8, 1).ravel() for i in ids[:123]])
    got = out.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got[:123 * g ** 3], want)
    assert (got[123 * g ** 3:] == 0xFFFFFFFF).all()


def test_small_batches_take_the_paired_kernel(csvlib, orc, cfg1):
    # untuned, a batch the paired front kernel takes at once runs paired;
    # larger batches and pools whose shape was set keep their shape, and the
    # paired and unpaired decodes agree
    torch = torch_cuda()
    vol, blob = cfg1
    pool = csvlib.Pool()
    pool.add_volume(blob)
    assert pool.shape_for(8)[0] == 2 and pool.shape_for(2048)[0] == 2
    assert pool.shape_for(1 << 16)[0] != 2
    ids = torch.tensor([5, 0, 7, 7, 2], dtype=torch.int32, device="cuda")
    a = torch.full((5 * 32768,), -1, dtype=torch.int32, device="cuda")
    b = torch.full_like(a, -1)
    log("small batch, library shape %s" % (pool.shape_for(5),))
    pool.decode(ids, a, lod=0)
    pool.set_shape((8, 3, 0, 0, 1))
    assert pool.shape_for(8)[0] == 8
    pool.decode(ids, b, lod=0)
    torch.cuda.synchronize()
    assert pool.last_error() == (0, 0)
    assert torch.equal(a, b)
    np.testing.assert_array_equal(a.cpu().numpy().view(np.uint32),
                                  orc.decode_bricks(blob, [5, 0, 7, 7, 2], [0] * 5))
