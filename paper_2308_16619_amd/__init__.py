"""MI355X compressed segmentation volumes: Python binding of libcsv.so.

Argument marshalling only: every step of brick decoding runs in the HIP
kernels behind the C ABI declared in include/csv.h.  PyTorch supplies device
memory and streams.  The library must be built (``build.py``); without it
every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsv.so")
# launch shapes tuned on an MI355X (csv_pool_tuning_load)
TUNING_PATH = os.path.join(HERE, "tuning_gfx950.txt")
BRICK = 32
MAX_LOD = 5

CSV_OK, CSV_EINVAL, CSV_ERANGE, CSV_ECORRUPT, CSV_ENOMEM, CSV_EHIP, CSV_EBUSY, CSV_EDETAIL = 0, -1, -2, -3, -4, -5, -6, -7
CSV_DETAIL_HOST = 1
_lib = None


class CsvError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        name = _lib.csv_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s: %s (%d)" % (what, name, code))
        self.code = code


class EncodeOpts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("brick_log2", "scale_bits", "lane_k", "lane_max", "sample_stride",
                                              "threads", "tables", "coding")]


class VolumeInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("nx", "ny", "nz", "brick_log2", "nbx", "nby", "nbz", "n_bricks",
                                              "scale_bits", "lane_k", "lane_max", "sample_stride")] + [
        ("freq", (ctypes.c_uint32 * 16) * 2), ("record_bytes", ctypes.c_uint64), ("blob_bytes", ctypes.c_uint64),
        ("coding", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Shape(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_int), ("groups_per_cu", ctypes.c_uint32), ("use_queue", ctypes.c_int),
                ("lpt_order", ctypes.c_int), ("chunks", ctypes.c_uint32), ("ms", ctypes.c_float)]

    def as_tuple(self):
        return (self.waves_per_group, self.groups_per_cu, self.use_queue, self.lpt_order, self.chunks)

    @classmethod
    def of(cls, shape):
        """(waves, groups, queue[, lpt[, chunks]]); lpt 0 and 1 chunk by default."""
        v = [int(x) for x in shape] + [0, 1][len(shape) - 3:] if len(shape) < 5 else [int(x) for x in shape]
        return cls(v[0], v[1], v[2], v[3], v[4], 0.0)


REQUEST_DTYPE = np.dtype([("brick_id", "<u4"), ("lod", "<u4"), ("tag", "<u8"), ("t_arrival_ns", "<u8")])
COMPLETION_DTYPE = np.dtype([("tag", "<u8"), ("brick_id", "<u4"), ("lod", "<u4"), ("data", "<u8"), ("elems", "<u4"),
                             ("status", "<i4"), ("hit", "<u4"), ("skipped", "<u4"), ("t_arrival_ns", "<u8"),
                             ("t_done_ns", "<u8")])


class FrameStats(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_uint32), ("requests", ctypes.c_uint32), ("distinct", ctypes.c_uint32),
                ("new_entries", ctypes.c_uint32), ("decoded", ctypes.c_uint32), ("hits", ctypes.c_uint32),
                ("evicted", ctypes.c_uint32), ("rebuilt", ctypes.c_uint32), ("used_bytes", ctypes.c_uint64),
                ("capacity_bytes", ctypes.c_uint64)]


class FrameDetailStats(ctypes.Structure):
    _fields_ = [("fallbacks", ctypes.c_uint32), ("wanted", ctypes.c_uint32), ("predicted", ctypes.c_uint32),
                ("staged", ctypes.c_uint32), ("released", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("uploaded_bytes", ctypes.c_uint64), ("resident_bytes", ctypes.c_uint64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("cache_bytes", ctypes.c_uint64), ("inflight_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_uint32),
                ("streams", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("requests", "hits", "misses", "joined", "completed", "batches",
                                              "evictions", "rebuilds", "decoded_bytes", "cache_bytes_used")] + [
        (n, ctypes.c_double) for n in ("p50_us", "p99_us", "p50_miss_us", "p99_miss_us", "max_us")] + [
        ("error", ctypes.c_int32), ("pad", ctypes.c_int32), ("worker_busy_ns", ctypes.c_uint64),
        ("worker_launch_ns", ctypes.c_uint64), ("stall_batch", ctypes.c_uint64), ("stall_inflight", ctypes.c_uint64),
        ("stall_slot", ctypes.c_uint64), ("skipped", ctypes.c_uint64), ("stall_staging", ctypes.c_uint64),
        ("detail_staged_bytes", ctypes.c_uint64), ("detail_releases", ctypes.c_uint64), ("failed", ctypes.c_uint64)]


class PoolInfo(ctypes.Structure):
    _fields_ = [("n_volumes", ctypes.c_uint32), ("n_bricks", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64),
                ("device", ctypes.c_int), ("brick_log2", ctypes.c_uint32), ("host_bytes", ctypes.c_uint64)]


def lib():
    """Load libcsv.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (binds the HIP runtime torch ships)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcsv.so is not built: run paper_2308_16619_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.csv_abi_version.restype = u32
        L.csv_strerror.restype = ctypes.c_char_p
        L.csv_strerror.argtypes = [i32]
        L.csv_encode_opts_default.argtypes = [ctypes.POINTER(EncodeOpts)]
        L.csv_encode_volume.argtypes = [vp, u32, u32, u32, ctypes.POINTER(EncodeOpts), ctypes.POINTER(vp),
                                        ctypes.POINTER(ctypes.c_size_t)]
        L.csv_encode_volume_gpu.argtypes = [vp, u32, u32, u32, ctypes.POINTER(EncodeOpts), i32, vp,
                                            ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]
        L.csv_encode_gpu_release.argtypes = [i32]
        L.csv_free.argtypes = [vp]
        L.csv_blob_info.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(VolumeInfo)]
        L.csv_blob_check.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(u32)]
        L.csv_pool_create.argtypes = [ctypes.POINTER(vp), i32]
        L.csv_pool_create_budget.argtypes = [ctypes.POINTER(vp), i32, u64]
        L.csv_pool_destroy.argtypes = [vp]
        L.csv_pool_add_volume.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(u32)]
        L.csv_pool_add_volume_ex.argtypes = [vp, vp, ctypes.c_size_t, u32, ctypes.POINTER(u32)]
        L.csv_pool_stage_detail.argtypes = [vp, vp, u32, vp, ctypes.POINTER(u32)]
        L.csv_pool_release_detail.argtypes = [vp, vp]
        L.csv_pool_set_detail_staging.argtypes = [vp, u64]
        L.csv_pool_info_get.argtypes = [vp, ctypes.POINTER(PoolInfo)]
        L.csv_output_elems.argtypes = [vp, u32, vp, ctypes.POINTER(u64)]
        L.csv_output_bytes.argtypes = [vp, u32, vp, ctypes.POINTER(u64)]
        L.csv_output_elems_log2.argtypes = [u32, vp, u32, vp, ctypes.POINTER(u64)]
        L.csv_decode_bricks_status.argtypes = [vp, vp, vp, u32, vp, u32, vp, vp, vp]
        L.csv_decode_bricks_devcount.argtypes = [vp, vp, vp, u32, vp, u32, vp, vp, vp]
        for f in ("csv_decode_bricks", "csv_decode_bricks_plain"):
            getattr(L, f).argtypes = [vp, vp, vp, u32, vp, u32, vp, vp]
        L.csv_decode_bricks_noalloc.argtypes = [vp, vp, vp, u32, vp, u32, vp, vp]
        L.csv_decode_bricks_shaped.argtypes = [vp, vp, vp, u32, vp, u32, vp, vp, ctypes.POINTER(Shape)]
        L.csv_pool_set_shape.argtypes = [vp, ctypes.POINTER(Shape)]
        L.csv_pool_tuning_save.argtypes = [vp, ctypes.c_char_p]
        L.csv_pool_shape_for.argtypes = [vp, vp, u32, u32, ctypes.POINTER(Shape)]
        L.csv_pool_tuning_load.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(u32)]
        L.csv_pool_get_shape.argtypes = [vp, ctypes.POINTER(Shape)]
        L.csv_bricks_visible.argtypes = [vp, vp, u32, vp, u32, vp, vp]
        L.csv_autotune.argtypes = [vp, vp, vp, u32, vp, u32, vp, vp, u32, ctypes.POINTER(Shape)]
        L.csv_graph_create.argtypes = [vp, vp, vp, u32, vp, u32, vp, vp, ctypes.POINTER(vp)]
        L.csv_graph_launch.argtypes = [vp, vp]
        L.csv_graph_destroy.argtypes = [vp]
        L.csv_pool_last_error.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(u32)]
        L.csv_now_ns.restype = u64
        L.csv_server_opts_default.argtypes = [ctypes.POINTER(ServerOpts)]
        L.csv_server_create.argtypes = [vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
        L.csv_server_submit.argtypes = [vp, vp, u32]
        L.csv_server_poll.argtypes = [vp, vp, u32, ctypes.POINTER(u32)]
        L.csv_server_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.csv_server_set_visible.argtypes = [vp, vp, u32]
        L.csv_server_reset_stats.argtypes = [vp]
        L.csv_server_read.argtypes = [vp, vp, vp]
        L.csv_server_cache_data.restype = vp
        L.csv_server_cache_data.argtypes = [vp]
        L.csv_server_run_trace.argtypes = [vp, vp, u32, vp, u64, ctypes.POINTER(u32)]
        L.csv_server_destroy.argtypes = [vp]
        L.csv_frame_cache_create.argtypes = [vp, u64, u32, ctypes.POINTER(vp)]
        L.csv_frame_cache_frame.argtypes = [vp, vp, vp, u32, vp, u32, vp, vp, ctypes.POINTER(FrameStats)]
        L.csv_frame_cache_data.restype = vp
        L.csv_frame_cache_data.argtypes = [vp]
        L.csv_frame_cache_frame_detail.argtypes = [vp, vp, vp, u32, vp, u32, vp, u32, vp, vp, vp,
                                                   ctypes.POINTER(FrameStats), ctypes.POINTER(FrameDetailStats)]
        L.csv_pool_detail_bytes.argtypes = [vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u64)]
        L.csv_frame_cache_read.argtypes = [vp, u64, u64, vp]
        L.csv_frame_cache_last_stats.argtypes = [vp, ctypes.POINTER(FrameStats)]
        L.csv_frame_cache_destroy.argtypes = [vp]
        if L.csv_abi_version() != 4:
            raise RuntimeError("libcsv.so ABI mismatch")
        _lib = L
    return _lib


def _chk(rc, what):
    if rc != CSV_OK:
        raise CsvError(rc, what)


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def encode_volume(vol: np.ndarray, brick_log2: int = 5, scale_bits: int = 10, lane_k: int = 64, lane_max: int = 64,
                  sample_stride: int = 0, threads: int = 0, tables: int = 2, coding: int = 0) -> bytes:
    """Compress a (nz, ny, nx) uint32 label volume into a container blob
    (tables: 2 rANS frequency tables, levels >= 1 and L_0, or 1 for all;
    coding: 0 interleaved rANS, 1 raw nibbles)."""
    L = lib()
    vol = np.ascontiguousarray(vol, dtype=np.uint32)
    nz, ny, nx = vol.shape
    o = EncodeOpts(brick_log2, scale_bits, lane_k, lane_max, sample_stride, threads, tables, coding)
    p = ctypes.c_void_p()
    n = ctypes.c_size_t()
    _chk(L.csv_encode_volume(_np_ptr(vol), nx, ny, nz, ctypes.byref(o), ctypes.byref(p), ctypes.byref(n)),
         "csv_encode_volume")
    try:
        return ctypes.string_at(p, n.value)
    finally:
        L.csv_free(p)


def encode_volume_gpu(vol, brick_log2: int = 5, scale_bits: int = 10, lane_k: int = 64, lane_max: int = 64,
                      sample_stride: int = 0, stream=None, tables: int = 2) -> bytes:
    """Compress a (nz, ny, nx) label volume on the GPU (same blob as
    encode_volume).  vol: a CUDA tensor of 4-byte labels (int32 or uint32
    bit patterns), or a numpy array, which is uploaded first."""
    import torch
    L = lib()
    if not isinstance(vol, torch.Tensor):
        vol = torch.from_numpy(np.ascontiguousarray(vol, dtype=np.uint32).view(np.int32)).cuda()
    if not vol.is_cuda or vol.dim() != 3 or vol.element_size() != 4:
        raise ValueError("vol must be a 3-d CUDA tensor of 4-byte labels")
    vol = vol.contiguous()
    nz, ny, nx = vol.shape
    o = EncodeOpts(brick_log2, scale_bits, lane_k, lane_max, sample_stride, 0, tables, 0)
    p = ctypes.c_void_p()
    n = ctypes.c_size_t()
    _chk(L.csv_encode_volume_gpu(ctypes.c_void_p(vol.data_ptr()), nx, ny, nz, ctypes.byref(o), vol.device.index or 0,
                                 _stream_handle(stream), ctypes.byref(p), ctypes.byref(n)), "csv_encode_volume_gpu")
    try:
        return ctypes.string_at(p, n.value)
    finally:
        L.csv_free(p)


def encode_gpu_release(device: int = 0) -> None:
    """Free the device buffers the GPU compressor keeps between calls."""
    _chk(lib().csv_encode_gpu_release(device), "csv_encode_gpu_release")


def blob_info(blob: bytes) -> dict:
    info = VolumeInfo()
    _chk(lib().csv_blob_info(blob, len(blob), ctypes.byref(info)), "csv_blob_info")
    d = {f: getattr(info, f) for f, _ in VolumeInfo._fields_ if f != "freq"}
    d["freq"] = np.array([[info.freq[t][s] for s in range(16)] for t in range(2)], dtype=np.uint32)
    return d


def blob_check(blob: bytes) -> tuple:
    """Validate every record of a container on the host: (CSV_OK or
    CSV_ECORRUPT / header error, first bad brick or None)."""
    bad = ctypes.c_uint32(0xFFFFFFFF)
    rc = lib().csv_blob_check(blob, len(blob), ctypes.byref(bad))
    return rc, (bad.value if rc == CSV_ECORRUPT and bad.value != 0xFFFFFFFF else None)


def output_offsets(lods, brick_log2: int = 5) -> tuple:
    """Element offsets of requests packed back to back, and the total
    (bricks of edge 2^brick_log2)."""
    lods = np.ascontiguousarray(lods, dtype=np.uint8)
    off = np.zeros(len(lods), dtype=np.uint64)
    tot = ctypes.c_uint64()
    _chk(lib().csv_output_elems_log2(brick_log2, _np_ptr(lods), len(lods), _np_ptr(off), ctypes.byref(tot)),
         "csv_output_elems_log2")
    return off, int(tot.value)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Pool:
    """Compressed volumes resident in HBM (one GPU)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self._p = ctypes.c_void_p()
        _chk(lib().csv_pool_create_budget(ctypes.byref(self._p), device, int(hbm_budget)), "csv_pool_create_budget")
        self.device = device

    def close(self):
        if self._p:
            lib().csv_pool_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_volume(self, blob: bytes, detail_host: bool = False) -> int:
        """Add one container; detail_host keeps level-0 detail in pinned host memory (Sec. 4.2)."""
        first = ctypes.c_uint32()
        if detail_host:
            _chk(lib().csv_pool_add_volume_ex(self._p, blob, len(blob), CSV_DETAIL_HOST, ctypes.byref(first)),
                 "csv_pool_add_volume_ex")
        else:
            _chk(lib().csv_pool_add_volume(self._p, blob, len(blob), ctypes.byref(first)), "csv_pool_add_volume")
        return first.value

    def stage_detail(self, ids_host, stream=None) -> int:
        """Upload the level-0 detail of host brick ids (in order, until the staging
        buffer is full); returns how many leading ids are ready for full-LOD decode."""
        a = np.ascontiguousarray(np.asarray(ids_host, dtype=np.uint32))
        done = ctypes.c_uint32()
        _chk(lib().csv_pool_stage_detail(self._p, a.ctypes.data if a.size else None, int(a.size),
                                         _stream_handle(stream), ctypes.byref(done)), "csv_pool_stage_detail")
        return done.value

    def release_detail(self, stream=None) -> None:
        _chk(lib().csv_pool_release_detail(self._p, _stream_handle(stream)), "csv_pool_release_detail")

    def detail_bytes(self, brick_id: int) -> int:
        """Staging bytes of a brick's level-0 detail (0: its record is whole in HBM)."""
        b = ctypes.c_uint32()
        _chk(lib().csv_pool_detail_bytes(self._p, int(brick_id), ctypes.byref(b), None), "csv_pool_detail_bytes")
        return b.value

    def set_detail_staging(self, nbytes: int) -> None:
        _chk(lib().csv_pool_set_detail_staging(self._p, int(nbytes)), "csv_pool_set_detail_staging")

    def info(self) -> dict:
        i = PoolInfo()
        _chk(lib().csv_pool_info_get(self._p, ctypes.byref(i)), "csv_pool_info_get")
        return {f: getattr(i, f) for f, _ in PoolInfo._fields_}

    def _args(self, ids, out, lods, lod, out_offsets, stream):
        return [self._p, ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(lods.data_ptr() if lods is not None else 0),
                lod, ctypes.c_void_p(out_offsets.data_ptr() if out_offsets is not None else 0), int(ids.numel()),
                ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)]

    def decode(self, ids, out, lods=None, lod=0, out_offsets=None, stream=None, plain: bool = False, shape=None,
               status=None):
        """Decode bricks `ids` (int32 cuda tensor) into `out` (int32 cuda
        tensor viewed as uint32).  `lods`: uint8 cuda tensor or None (all at
        `lod`); `out_offsets`: int64 cuda tensor of element offsets (needed
        with `lods`) or None (request i at i * (32 >> lod)^3).  `plain`: one
        launch per brick.  `shape`: (waves_per_group, groups_per_cu,
        use_queue[, lpt_order]) launch shape; default: the pool's shape.
        `status`: int32 cuda tensor of ids.numel() zeros; failed requests
        get their error code (csv_decode_bricks_status)."""
        args = self._args(ids, out, lods, lod, out_offsets, stream)
        if status is not None:
            _chk(lib().csv_decode_bricks_status(*args, ctypes.c_void_p(status.data_ptr())), "csv_decode_bricks_status")
        elif shape is not None:
            sh = Shape.of(shape)
            _chk(lib().csv_decode_bricks_shaped(*args, ctypes.byref(sh)), "csv_decode_bricks_shaped")
        elif plain:
            _chk(lib().csv_decode_bricks_plain(*args), "csv_decode_bricks_plain")
        else:
            _chk(lib().csv_decode_bricks(*args), "csv_decode_bricks")

    def decode_devcount(self, ids, out, n_dev, lods=None, lod=0, out_offsets=None, stream=None):
        """decode() of requests 0 .. min(ids.numel(), n_dev[0]) - 1, the count
        read on the device from `n_dev` (int32/uint32 cuda tensor) by the
        kernels (csv_decode_bricks_devcount); nothing waits for the device."""
        a = self._args(ids, out, lods, lod, out_offsets, stream)
        _chk(lib().csv_decode_bricks_devcount(*a[:6], ctypes.c_void_p(n_dev.data_ptr()), *a[6:]),
             "csv_decode_bricks_devcount")

    def decode_noalloc(self, ids, out, lods=None, lod=0, out_offsets=None, stream=None):
        """decode() through csv_decode_bricks_noalloc: no device allocation;
        the library's fixed scratch array on the device is shared by every
        call on that GPU, so calls must not overlap."""
        _chk(lib().csv_decode_bricks_noalloc(*self._args(ids, out, lods, lod, out_offsets, stream)),
             "csv_decode_bricks_noalloc")

    def visible(self, ids, visible_bits, n_label_bits: int, out=None, stream=None):
        """Empty-space test: out[i] = 1 if some label of brick ids[i] has its
        bit set in `visible_bits` (int32 cuda tensor, bit label & 31 of word
        label >> 5; labels >= n_label_bits are invisible), else 0.  `out`:
        uint8 cuda tensor of ids.numel() entries, allocated if None.
        Returns out (asynchronous on the stream)."""
        if out is None:
            import torch
            out = torch.empty(ids.numel(), dtype=torch.uint8, device=ids.device)
        bits = visible_bits.data_ptr() if (visible_bits is not None and n_label_bits) else 0
        _chk(lib().csv_bricks_visible(self._p, ctypes.c_void_p(ids.data_ptr()), int(ids.numel()),
                                      ctypes.c_void_p(bits), int(n_label_bits), ctypes.c_void_p(out.data_ptr()),
                                      _stream_handle(stream)), "csv_bricks_visible")
        return out

    def set_shape(self, shape):
        sh = Shape.of(shape)
        _chk(lib().csv_pool_set_shape(self._p, ctypes.byref(sh)), "csv_pool_set_shape")

    def get_shape(self):
        sh = Shape()
        _chk(lib().csv_pool_get_shape(self._p, ctypes.byref(sh)), "csv_pool_get_shape")
        return sh.as_tuple()

    def autotune(self, ids, out, lods=None, lod=0, out_offsets=None, stream=None, reps: int = 3):
        """Time every launch shape on this request set; the fastest becomes
        the pool's shape.  Returns (shape tuple, ms per launch)."""
        sh = Shape()
        _chk(lib().csv_autotune(*self._args(ids, out, lods, lod, out_offsets, stream), reps, ctypes.byref(sh)),
             "csv_autotune")
        return sh.as_tuple(), sh.ms

    def shape_for(self, n: int, lod: int = 0, per_request_lods: bool = False, with_ms: bool = False):
        """The launch shape a decode of n requests would use (with_ms: also
        its tuned time per call, 0 for the pool's untuned shape)."""
        sh = Shape()
        _chk(lib().csv_pool_shape_for(self._p, ctypes.c_void_p(1 if per_request_lods else 0), lod, n,
                                      ctypes.byref(sh)), "csv_pool_shape_for")
        return (sh.as_tuple(), sh.ms) if with_ms else sh.as_tuple()

    def save_tuning(self, path: str) -> None:
        """Write the pool's tuned shapes (by request-set class) to a text file."""
        _chk(lib().csv_pool_tuning_save(self._p, os.fsencode(path)), "csv_pool_tuning_save")

    def load_tuning(self, path: str = None) -> int:
        """Add the tuned shapes of a file made on the same kind of device
        (default: the file shipped for gfx950); returns how many were added."""
        got = ctypes.c_uint32(0)
        _chk(lib().csv_pool_tuning_load(self._p, os.fsencode(path or TUNING_PATH), ctypes.byref(got)),
             "csv_pool_tuning_load")
        return int(got.value)

    def graph(self, ids, out, lods=None, lod=0, out_offsets=None, stream=None):
        """Capture this decode into a replayable HIP graph."""
        return Graph(self, self._args(ids, out, lods, lod, out_offsets, stream))

    def last_error(self):
        code = ctypes.c_int()
        bid = ctypes.c_uint32()
        _chk(lib().csv_pool_last_error(self._p, ctypes.byref(code), ctypes.byref(bid)), "csv_pool_last_error")
        return code.value, bid.value


class Graph:
    """A decode captured once and replayed with csv_graph_launch."""

    def __init__(self, pool, args):
        self._g = ctypes.c_void_p()
        self._pool = pool  # keep the pool alive
        _chk(lib().csv_graph_create(*args, ctypes.byref(self._g)), "csv_graph_create")

    def launch(self, stream=None):
        _chk(lib().csv_graph_launch(self._g, _stream_handle(stream)), "csv_graph_launch")

    def close(self):
        if self._g:
            lib().csv_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now_ns() -> int:
    return int(lib().csv_now_ns())


class Server:
    """Serving loop over a pool: submit requests, poll completions."""

    def __init__(self, pool, cache_bytes=1 << 30, inflight_bytes=256 << 20, max_batch=4096, streams=4):
        o = ServerOpts(cache_bytes, inflight_bytes, max_batch, streams)
        self._s = ctypes.c_void_p()
        self._pool = pool
        _chk(lib().csv_server_create(pool._p, ctypes.byref(o), ctypes.byref(self._s)), "csv_server_create")

    @staticmethod
    def requests(brick_ids, lods, tags=None, t_arrival_ns=None) -> np.ndarray:
        n = len(brick_ids)
        r = np.zeros(n, dtype=REQUEST_DTYPE)
        r["brick_id"] = brick_ids
        r["lod"] = lods
        r["tag"] = np.arange(n) if tags is None else tags
        r["t_arrival_ns"] = now_ns() if t_arrival_ns is None else t_arrival_ns
        return r

    def submit(self, reqs: np.ndarray):
        reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        _chk(lib().csv_server_submit(self._s, _np_ptr(reqs), len(reqs)), "csv_server_submit")

    def poll(self, cap: int = 65536) -> np.ndarray:
        buf = np.zeros(cap, dtype=COMPLETION_DTYPE)
        got = ctypes.c_uint32()
        _chk(lib().csv_server_poll(self._s, _np_ptr(buf), cap, ctypes.byref(got)), "csv_server_poll")
        return buf[:got.value]

    def read(self, completion) -> np.ndarray:
        """The decoded brick of one completion (valid until the next poll)."""
        c = np.ascontiguousarray(np.asarray(completion, dtype=COMPLETION_DTYPE).reshape(1))
        out = np.zeros(int(c["elems"][0]), dtype=np.uint32)
        _chk(lib().csv_server_read(self._s, _np_ptr(c), _np_ptr(out)), "csv_server_read")
        return out

    def cache_ptr(self) -> int:
        """Device address of the decoded-brick cache (completions point into it)."""
        return int(lib().csv_server_cache_data(self._s) or 0)

    def run_trace(self, reqs: np.ndarray, collect: bool = False, timeout_s: float = 10.0):
        reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        done = np.zeros(len(reqs), dtype=COMPLETION_DTYPE) if collect else None
        got = ctypes.c_uint32()
        rc = lib().csv_server_run_trace(self._s, _np_ptr(reqs), len(reqs),
                                        _np_ptr(done) if collect else ctypes.c_void_p(0), int(timeout_s * 1e9),
                                        ctypes.byref(got))
        if rc not in (CSV_OK, CSV_EBUSY):
            _chk(rc, "csv_server_run_trace")
        return (done[:got.value] if collect else None), got.value

    def stats(self) -> dict:
        st = Stats()
        _chk(lib().csv_server_stats(self._s, ctypes.byref(st)), "csv_server_stats")
        return {f: getattr(st, f) for f, _ in Stats._fields_}

    def reset_stats(self):
        _chk(lib().csv_server_reset_stats(self._s), "csv_server_reset_stats")

    def set_visible(self, visible):
        """Visibility table (uint8 per global brick id, host) or None: requests
        for bricks whose byte is 0 complete at once as skipped."""
        if visible is None:
            _chk(lib().csv_server_set_visible(self._s, ctypes.c_void_p(0), 0), "csv_server_set_visible")
            return
        v = np.ascontiguousarray(visible, dtype=np.uint8)
        _chk(lib().csv_server_set_visible(self._s, _np_ptr(v), len(v)), "csv_server_set_visible")

    def close(self):
        if self._s:
            lib().csv_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FrameCache:
    """Per-frame cache of decoded bricks on the GPU (free stacks per LOD, a
    top pointer, rebuild on overflow)."""

    def __init__(self, pool, cache_bytes: int, max_requests: int):
        self._c = ctypes.c_void_p()
        self._pool = pool
        self.max_requests = max_requests
        _chk(lib().csv_frame_cache_create(pool._p, int(cache_bytes), int(max_requests), ctypes.byref(self._c)),
             "csv_frame_cache_create")

    def frame(self, ids, lods, visible_bits=None, n_label_bits: int = 0, slots=None, stream=None,
              stats: bool = True):
        """ids (int32/uint32 CUDA tensor), lods (uint8 CUDA tensor); returns
        (slots int64 CUDA tensor: element offsets in data(), -1 if not stored,
        stats dict).  stats=False: nothing waits for the device and the dict
        is None (last_stats() reads it later)."""
        import torch
        n = ids.numel()
        if slots is None:
            slots = torch.empty(n, dtype=torch.int64, device=ids.device)
        st = FrameStats()
        vb = ctypes.c_void_p(visible_bits.data_ptr()) if visible_bits is not None else None
        _chk(lib().csv_frame_cache_frame(self._c, ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(lods.data_ptr()),
                                         n, vb, int(n_label_bits), ctypes.c_void_p(slots.data_ptr()),
                                         _stream_handle(stream), ctypes.byref(st) if stats else None),
             "csv_frame_cache_frame")
        return slots, ({f: getattr(st, f) for f, _ in FrameStats._fields_} if stats else None)

    def frame_detail(self, ids, lods, predict=None, visible_bits=None, n_label_bits: int = 0, slots=None,
                     served=None, stream=None, stats: bool = True):
        """A frame on a pool with level-0 detail in host memory: full-LOD
        requests without detail on the device are served at LOD 1 and their
        detail uploaded for the next frame, with the detail of `predict`
        (int32/uint32 CUDA tensor of brick ids, most urgent first).  Returns
        (slots, served LODs uint8 CUDA tensor, stats dict, detail stats
        dict); both dicts are None with stats=False."""
        import torch
        n = ids.numel()
        if slots is None:
            slots = torch.empty(n, dtype=torch.int64, device=ids.device)
        if served is None:
            served = torch.empty(n, dtype=torch.uint8, device=ids.device)
        st, ds = FrameStats(), FrameDetailStats()
        vb = ctypes.c_void_p(visible_bits.data_ptr()) if visible_bits is not None else None
        npred = predict.numel() if predict is not None else 0
        pp = ctypes.c_void_p(predict.data_ptr()) if npred else None
        _chk(lib().csv_frame_cache_frame_detail(
            self._c, ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(lods.data_ptr()), n, vb, int(n_label_bits),
            pp, npred, ctypes.c_void_p(slots.data_ptr()), ctypes.c_void_p(served.data_ptr()), _stream_handle(stream),
            ctypes.byref(st) if stats else None, ctypes.byref(ds) if stats else None), "csv_frame_cache_frame_detail")
        if not stats:
            return slots, served, None, None
        return (slots, served, {f: getattr(st, f) for f, _ in FrameStats._fields_},
                {f: getattr(ds, f) for f, _ in FrameDetailStats._fields_ if f != "pad"})

    def last_stats(self):
        """Statistics of the last frame (waits for the device); raises
        CsvError(CSV_ENOMEM) if that frame did not fit."""
        st = FrameStats()
        _chk(lib().csv_frame_cache_last_stats(self._c, ctypes.byref(st)), "csv_frame_cache_last_stats")
        return {f: getattr(st, f) for f, _ in FrameStats._fields_}

    def data_ptr(self) -> int:
        """Device address of the cache memory (uint32 labels)."""
        return lib().csv_frame_cache_data(self._c)

    def read(self, elem_offset: int, n: int) -> np.ndarray:
        """Copy n labels from the cache, starting at elem_offset, to host memory."""
        out = np.empty(n, dtype=np.uint32)
        _chk(lib().csv_frame_cache_read(self._c, int(elem_offset), int(n), _np_ptr(out)), "csv_frame_cache_read")
        return out

    def close(self):
        if self._c:
            lib().csv_frame_cache_destroy(self._c)
            self._c = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
