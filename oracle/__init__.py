"""ORACLE -- test infrastructure only.

A plain CPU implementation of compressed segmentation volumes, written from
the paper (Piochowiak & Dachsbacher, IEEE TVCG 2023): resolution pyramid
(Sec. 3.1), brick encoding (Sec. 3.2, Alg. 2), two static frequency tables
and rANS (Sec. 3.3), decoding to a level of detail (Sec. 3.4, Alg. 1).  The
arithmetic lives in ``csv_oracle.c``; this module only marshals arguments.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the GPU library.

Parity status per function (what pins it, see tests/test_oracle_*.py):
  pyramid          brute-force definition (mode of 8, first-occurrence ties)
  brick_symbols    hand-worked golden bricks; brute-force first-applicable
                   operation on 4^3 bricks; decode(LOD t) == pyramid level t
  normalize_table  closed-form invariants (sum, floor, +1 smoothing)
  rans_*           closed form for a uniform table; state invariants;
                   size bound; exact round trip
  encode/decode    round trip identity on every brick; LOD t equals the
                   pyramid level computed from the definition
The compressed bytes themselves are not fixed by the paper (parity
unpinned for the byte layout: it is this project's format).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csv_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

# operation codes (position in the encoder's test order)
RP, RX, RY, RZ, P0, PD, PA = range(7)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        u32, u64 = ctypes.c_uint32, ctypes.c_uint64
        L.orc_encode_volume.argtypes = [vp, u32, u32, u32, u32, u32, u32, u32, u32, u32,
                                        ctypes.POINTER(vp), ctypes.POINTER(u64), vp]
        L.orc_decode_brick.argtypes = [vp, u64, u32, u32, vp]
        L.orc_decode_bricks.argtypes = [vp, u64, vp, vp, u32, vp]
        L.orc_volume_info.argtypes = [vp, u64, vp]
        L.orc_pyramid.argtypes = [vp, u32, vp, vp]
        L.orc_brick_symbols.argtypes = [vp, u32, vp, u32, vp, vp, vp, u32, vp]
        L.orc_replay.argtypes = [vp, vp, u32, vp, u32, u32, vp]
        L.orc_normalize_table.argtypes = [vp, u32, vp]
        L.orc_rans_encode.argtypes = [vp, u32, u32, u32, vp, u32, vp, vp, vp]
        L.orc_rans_decode.argtypes = [vp, u32, vp, u32, u32, vp, u32, u32, vp, vp]
        L.orc_free.argtypes = [vp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


class OracleError(RuntimeError):
    def __init__(self, rc):
        super().__init__("oracle error %d" % rc)
        self.rc = rc


def _chk(rc):
    if rc != 0:
        raise OracleError(rc)


def num_threads() -> int:
    """Host threads the oracle's parallel loops (over bricks) use."""
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Host threads for the oracle's later parallel loops."""
    _load().orc_set_threads(int(n))


# ---------------------------------------------------------------- volume --
def encode_volume(vol: np.ndarray, brick_log2: int = 5, scale_bits: int = 12, lane_k: int = 256,
                  lane_max: int = 64, sample_stride: int = 0, return_hist: bool = False, tables: int = 2):
    """Encode a (nz, ny, nx) uint32 volume; returns the container bytes.
    tables: 2 frequency tables (levels >= 1, L_0), 1 for all symbols, or 0
    for no entropy coding (raw nibbles)."""
    vol = np.ascontiguousarray(vol, dtype=np.uint32)
    nz, ny, nx = vol.shape
    blob = ctypes.c_void_p()
    nbytes = ctypes.c_uint64()
    hist = np.zeros(8, dtype=np.uint64)
    _chk(_load().orc_encode_volume(_p(vol), nx, ny, nz, brick_log2, scale_bits, lane_k, lane_max, sample_stride,
                                   tables, ctypes.byref(blob), ctypes.byref(nbytes), _p(hist)))
    out = ctypes.string_at(blob, nbytes.value)
    _load().orc_free(blob)
    return (out, hist) if return_hist else out


def volume_info(blob: bytes) -> dict:
    a = np.frombuffer(blob, dtype=np.uint8)
    info = np.zeros(16, dtype=np.uint32)
    _chk(_load().orc_volume_info(_p(a), len(blob), _p(info)))
    keys = ["magic", "version", "nx", "ny", "nz", "brick_log2", "nbx", "nby", "nbz", "n_bricks", "scale_bits",
            "lane_k", "lane_max", "sample_stride"]
    d = {k: int(info[i]) for i, k in enumerate(keys)}
    freq = np.frombuffer(blob, dtype=np.uint16, count=32, offset=64).reshape(2, 16)
    d["freq"] = freq.astype(np.uint32)
    return d


def decode_brick(blob: bytes, brick_id: int, lod: int = 0) -> np.ndarray:
    """Decode one brick to LOD `lod`; returns (g, g, g) labels, g = b >> lod."""
    info = volume_info(blob)
    g = (1 << info["brick_log2"]) >> lod
    out = np.zeros((g, g, g), dtype=np.uint32)
    a = np.frombuffer(blob, dtype=np.uint8)
    _chk(_load().orc_decode_brick(_p(a), len(blob), brick_id, lod, _p(out)))
    return out


def decode_bricks(blob: bytes, ids, lods) -> np.ndarray:
    """Decode many requests; outputs packed back to back in request order."""
    info = volume_info(blob)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    lods = np.ascontiguousarray(np.broadcast_to(np.asarray(lods, dtype=np.uint8), ids.shape))
    N = info["brick_log2"]
    total = int(sum(8 ** (N - int(t)) for t in lods))
    out = np.zeros(total, dtype=np.uint32)
    a = np.frombuffer(blob, dtype=np.uint8)
    _chk(_load().orc_decode_bricks(_p(a), len(blob), _p(ids), _p(lods), len(ids), _p(out)))
    return out


# ------------------------------------------------------------ the steps --
def pyramid(brick: np.ndarray):
    """Levels L_0..L_N of one brick, each a Morton-ordered array, plus the
    constant-subtree flags."""
    brick = np.ascontiguousarray(brick, dtype=np.uint32)
    b = brick.shape[0]
    N = b.bit_length() - 1
    tot = sum(8 ** (N - l) for l in range(N + 1))
    lab = np.zeros(tot, dtype=np.uint32)
    cst = np.zeros(tot, dtype=np.uint8)
    _chk(_load().orc_pyramid(_p(brick), N, _p(lab), _p(cst)))
    levels, consts, o = [], [], 0
    for l in range(N + 1):
        n = 8 ** (N - l)
        levels.append(lab[o:o + n].copy())
        consts.append(cst[o:o + n].astype(bool))
        o += n
    return levels, consts


def brick_symbols(brick: np.ndarray):
    """Alg. 2 output of one brick: (symbols, cum, palette).  cum[m] is the
    number of symbols through the segment of child level m."""
    brick = np.ascontiguousarray(brick, dtype=np.uint32)
    b = brick.shape[0]
    N = b.bit_length() - 1
    cap = 2 * b ** 3 + 64
    sym = np.zeros(cap, dtype=np.uint8)
    cum = np.zeros(N, dtype=np.uint32)
    pal = np.zeros(cap, dtype=np.uint32)
    n = ctypes.c_uint32()
    npal = ctypes.c_uint32()
    _chk(_load().orc_brick_symbols(_p(brick), N, _p(sym), cap, ctypes.byref(n), _p(cum), _p(pal), cap,
                                   ctypes.byref(npal)))
    return sym[:n.value].copy(), cum, pal[:npal.value].copy()


def replay(sym: np.ndarray, cum, palette: np.ndarray, brick_log2: int, lod: int = 0) -> np.ndarray:
    """Alg. 1 on an explicit symbol stream; returns the dense LOD block."""
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    if sym.size == 0:
        sym = np.zeros(1, dtype=np.uint8)
    cum = np.ascontiguousarray(cum, dtype=np.uint32)
    palette = np.ascontiguousarray(palette, dtype=np.uint32)
    g = (1 << brick_log2) >> lod
    out = np.zeros((g, g, g), dtype=np.uint32)
    _chk(_load().orc_replay(_p(sym), _p(cum), brick_log2, _p(palette), len(palette), lod, _p(out)))
    return out


def normalize_table(counts, scale_bits: int = 12) -> np.ndarray:
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    f = np.zeros(16, dtype=np.uint32)
    _chk(_load().orc_normalize_table(_p(c), scale_bits, _p(f)))
    return f


def rans_encode(sym, freq2x16, scale_bits: int = 12, lanes: int = 1, tab_split=None):
    """Interleaved rANS over explicit symbols; returns (states, words)."""
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    n = len(sym)
    if tab_split is None:
        tab_split = n
    f = np.ascontiguousarray(freq2x16, dtype=np.uint32).reshape(2, 16)
    st = np.zeros(lanes, dtype=np.uint32)
    w = np.zeros(n + 16, dtype=np.uint16)
    nw = ctypes.c_uint32()
    _chk(_load().orc_rans_encode(_p(sym if n else np.zeros(1, np.uint8)), n, tab_split, lanes, _p(f), scale_bits,
                                 _p(st), _p(w), ctypes.byref(nw)))
    return st, w[:nw.value].copy()


def rans_decode(states, words, n: int, freq2x16, scale_bits: int = 12, tab_split=None):
    """Returns (symbols, final states, words consumed)."""
    st = np.array(states, dtype=np.uint32)
    words = np.ascontiguousarray(words, dtype=np.uint16)
    if tab_split is None:
        tab_split = n
    f = np.ascontiguousarray(freq2x16, dtype=np.uint32).reshape(2, 16)
    sym = np.zeros(max(n, 1), dtype=np.uint8)
    cur = ctypes.c_uint32()
    _chk(_load().orc_rans_decode(_p(st), len(st), _p(words if len(words) else np.zeros(1, np.uint16)), len(words),
                                 tab_split, _p(f), scale_bits, n, _p(sym), ctypes.byref(cur)))
    return sym[:n], st, cur.value
