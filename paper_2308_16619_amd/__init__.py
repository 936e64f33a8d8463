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
BRICK = 32
MAX_LOD = 5

CSV_OK, CSV_EINVAL, CSV_ERANGE, CSV_ECORRUPT, CSV_ENOMEM, CSV_EHIP, CSV_EBUSY = 0, -1, -2, -3, -4, -5, -6
_lib = None


class CsvError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        name = _lib.csv_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s: %s (%d)" % (what, name, code))
        self.code = code


class EncodeOpts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("brick_log2", "scale_bits", "lane_k", "lane_max", "sample_stride",
                                              "threads")]


class VolumeInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("nx", "ny", "nz", "brick_log2", "nbx", "nby", "nbz", "n_bricks",
                                              "scale_bits", "lane_k", "lane_max", "sample_stride")] + [
        ("freq", (ctypes.c_uint32 * 16) * 2), ("record_bytes", ctypes.c_uint64), ("blob_bytes", ctypes.c_uint64)]


class PoolInfo(ctypes.Structure):
    _fields_ = [("n_volumes", ctypes.c_uint32), ("n_bricks", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64),
                ("device", ctypes.c_int)]


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
        L.csv_free.argtypes = [vp]
        L.csv_blob_info.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(VolumeInfo)]
        L.csv_pool_create.argtypes = [ctypes.POINTER(vp), i32]
        L.csv_pool_destroy.argtypes = [vp]
        L.csv_pool_add_volume.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(u32)]
        L.csv_pool_info_get.argtypes = [vp, ctypes.POINTER(PoolInfo)]
        L.csv_output_elems.argtypes = [vp, u32, vp, ctypes.POINTER(u64)]
        for f in ("csv_decode_bricks", "csv_decode_bricks_plain"):
            getattr(L, f).argtypes = [vp, vp, vp, u32, vp, u32, vp, vp]
        L.csv_pool_last_error.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(u32)]
        if L.csv_abi_version() != 1:
            raise RuntimeError("libcsv.so ABI mismatch")
        _lib = L
    return _lib


def _chk(rc, what):
    if rc != CSV_OK:
        raise CsvError(rc, what)


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def encode_volume(vol: np.ndarray, brick_log2: int = 5, scale_bits: int = 10, lane_k: int = 64, lane_max: int = 64,
                  sample_stride: int = 0, threads: int = 0) -> bytes:
    """Compress a (nz, ny, nx) uint32 label volume into a container blob."""
    L = lib()
    vol = np.ascontiguousarray(vol, dtype=np.uint32)
    nz, ny, nx = vol.shape
    o = EncodeOpts(brick_log2, scale_bits, lane_k, lane_max, sample_stride, threads)
    p = ctypes.c_void_p()
    n = ctypes.c_size_t()
    _chk(L.csv_encode_volume(_np_ptr(vol), nx, ny, nz, ctypes.byref(o), ctypes.byref(p), ctypes.byref(n)),
         "csv_encode_volume")
    try:
        return ctypes.string_at(p, n.value)
    finally:
        L.csv_free(p)


def blob_info(blob: bytes) -> dict:
    info = VolumeInfo()
    _chk(lib().csv_blob_info(blob, len(blob), ctypes.byref(info)), "csv_blob_info")
    d = {f: getattr(info, f) for f, _ in VolumeInfo._fields_ if f != "freq"}
    d["freq"] = np.array([[info.freq[t][s] for s in range(16)] for t in range(2)], dtype=np.uint32)
    return d


def output_offsets(lods) -> tuple:
    """Element offsets of requests packed back to back, and the total."""
    lods = np.ascontiguousarray(lods, dtype=np.uint8)
    off = np.zeros(len(lods), dtype=np.uint64)
    tot = ctypes.c_uint64()
    _chk(lib().csv_output_elems(_np_ptr(lods), len(lods), _np_ptr(off), ctypes.byref(tot)), "csv_output_elems")
    return off, int(tot.value)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Pool:
    """Compressed volumes resident in HBM (one GPU)."""

    def __init__(self, device: int = 0):
        self._p = ctypes.c_void_p()
        _chk(lib().csv_pool_create(ctypes.byref(self._p), device), "csv_pool_create")
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

    def add_volume(self, blob: bytes) -> int:
        first = ctypes.c_uint32()
        _chk(lib().csv_pool_add_volume(self._p, blob, len(blob), ctypes.byref(first)), "csv_pool_add_volume")
        return first.value

    def info(self) -> dict:
        i = PoolInfo()
        _chk(lib().csv_pool_info_get(self._p, ctypes.byref(i)), "csv_pool_info_get")
        return {f: getattr(i, f) for f, _ in PoolInfo._fields_}

    def decode(self, ids, out, lods=None, lod=0, out_offsets=None, stream=None, plain: bool = False):
        """Decode bricks `ids` (int32 cuda tensor) into `out` (int32 cuda
        tensor viewed as uint32).  `lods`: uint8 cuda tensor or None (all at
        `lod`); `out_offsets`: int64 cuda tensor of element offsets (needed
        with `lods`) or None (request i at i * (32 >> lod)^3)."""
        fn = lib().csv_decode_bricks_plain if plain else lib().csv_decode_bricks
        n = int(ids.numel())
        _chk(fn(self._p, ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(lods.data_ptr() if lods is not None else 0),
                lod, ctypes.c_void_p(out_offsets.data_ptr() if out_offsets is not None else 0), n,
                ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "csv_decode_bricks")

    def last_error(self):
        code = ctypes.c_int()
        bid = ctypes.c_uint32()
        _chk(lib().csv_pool_last_error(self._p, ctypes.byref(code), ctypes.byref(bid)), "csv_pool_last_error")
        return code.value, bid.value
