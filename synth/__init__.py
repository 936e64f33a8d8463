"""Seeded synthetic label volumes (inputs for tests and the benchmark).

The volumes stand in for the paper's Cells, Fiber and Cortex data sets
(Section 5), which are not available here.  This module holds no part of the
compression method: it only generates labels.  The generators are plain C
(``synth.c``) driven through ctypes; volumes are numpy uint32 arrays of shape
(nz, ny, nx), x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile synth.c into libsynth.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.synth_voronoi_bg.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64]
        lib.synth_cells.argtypes = [u32p, u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64]
        lib.synth_blobs.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64]
        lib.synth_neurite.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        d, u64, u32, vp = ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        lib.synth_camera_trace.argtypes = [u32, u32, u32, d, d, d, u64, u64, d, d, d, d, u32, u32, u64, vp, vp, vp,
                                           ctypes.POINTER(u64)]
        lib.synth_camera_path.argtypes = [u32, u32, u32, u64, vp]
        lib.synth_camera_pose.argtypes = [vp, d, vp, vp]
        lib.synth_camera_pose.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def voronoi_bg(n: int = 64, sites: int = 200, bg: float = 0.30, seed: int = 1) -> np.ndarray:
    """Voronoi of `sites` uniform sites, labels 1..sites, then whole sites
    cleared to 0 in seeded order until >= bg of the voxels are 0."""
    out = np.empty((n, n, n), dtype=np.uint32)
    rc = _load().synth_voronoi_bg(_ptr(out), n, sites, bg, seed)
    assert rc == 0, rc
    return out


def cells(n: int = 512, grid: int = 37, p_noise: float = 0.5, seed: int = 2) -> np.ndarray:
    """Jittered-grid Voronoi of grid^3 cells with 1-voxel boundary noise."""
    out = np.empty((n, n, n), dtype=np.uint32)
    tmp = np.empty((n, n, n), dtype=np.uint32)
    rc = _load().synth_cells(_ptr(out), _ptr(tmp), n, grid, p_noise, seed)
    assert rc == 0, rc
    return out


def blobs(n: int = 512, sites: int = 50, amp: float = 24.0, seed: int = 4) -> np.ndarray:
    """Voronoi of `sites` sites over a smoothly warped space (large blobs)."""
    out = np.empty((n, n, n), dtype=np.uint32)
    rc = _load().synth_blobs(_ptr(out), n, sites, amp, seed)
    assert rc == 0, rc
    return out


# fraction of the volume given to tubes before overlaps; chosen so that about
# 45 % of the voxels stay background 0 at the default density
NEURITE_FILL = 1.45


def neurite(nx: int = 1024, ny: int = 1024, nz: int = 1024, labels: int = 20000, fill: float = NEURITE_FILL,
            seed: int = 3) -> np.ndarray:
    """Branching random-walk tubes of radius 2..8 with Zipf sizes."""
    out = np.empty((nz, ny, nx), dtype=np.uint32)
    painted = ctypes.c_uint64(0)
    rc = _load().synth_neurite(_ptr(out), nx, ny, nz, labels, fill, seed, ctypes.byref(painted))
    assert rc == 0, rc
    return out


def random_brick(b: int, n_labels: int, seed: int, smooth: int = 0) -> np.ndarray:
    """A b^3 brick of labels 1..n_labels for property tests: i.i.d. labels,
    optionally smoothed by repeated majority copying from a random axis
    neighbour so that the brick has regions of equal labels."""
    rng = np.random.default_rng(seed)
    a = rng.integers(1, n_labels + 1, size=(b, b, b), dtype=np.uint32)
    for _ in range(smooth):
        ax = int(rng.integers(0, 3))
        sh = np.roll(a, 1, axis=ax)
        take = rng.random(a.shape) < 0.6
        a = np.where(take, sh, a).astype(np.uint32)
    return a



def camera_trace(nx: int, ny: int, nz: int, rate: float, duration_s: float, seed: int = 6, path_seed: int = 7,
                 period_s: float = 20.0, cone_deg: float = 60.0, d_max: float = 3000.0, d0: float = 1663.0,
                 brick: int = 32, max_lod: int = 2, t0_s: float = 0.0):
    """Brick requests of a camera fly-through, as a renderer issues them:
    Poisson arrivals at `rate` per second over [t0_s, t0_s + duration_s), a
    camera on a closed Catmull-Rom path (one lap per period_s) looking along
    its tangent, each request a point in the view cone with distance density
    proportional to d^2 up to d_max, at level of detail 0 below d0 and
    floor(log2(d / d0)) + 1 (at most max_lod) beyond.  Returns (brick ids
    u32 with x fastest, lods u8, arrival times in ns relative to t0_s)."""
    cap = int(rate * duration_s * 1.2) + 1024
    ids = np.empty(cap, np.uint32)
    lods = np.empty(cap, np.uint8)
    t = np.empty(cap, np.uint64)
    n = ctypes.c_uint64()
    lib = _load()
    rc = lib.synth_camera_trace(nx, ny, nz, float(rate), float(duration_s), float(t0_s), seed, path_seed,
                                float(period_s), float(cone_deg), float(d_max), float(d0), brick, max_lod, cap,
                                ids.ctypes.data_as(ctypes.c_void_p), lods.ctypes.data_as(ctypes.c_void_p),
                                t.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n))
    assert rc == 0, rc
    k = n.value
    return ids[:k].copy(), lods[:k].copy(), t[:k].copy()


def camera_path(nx: int, ny: int, nz: int, seed: int = 7) -> np.ndarray:
    """The 8 control points (x, y, z) of camera_trace's path (path_seed)."""
    c = np.empty((8, 3), np.float64)
    assert _load().synth_camera_path(nx, ny, nz, seed, c.ctypes.data_as(ctypes.c_void_p)) == 0
    return c


def camera_pose(ctrl: np.ndarray, u):
    """Camera position and path tangent at parameters u in [0, 1)."""
    ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    pos, tan = np.empty((len(u), 3)), np.empty((len(u), 3))
    lib, cp = _load(), ctrl.ctypes.data_as(ctypes.c_void_p)
    p3, t3 = np.empty(3), np.empty(3)
    for i, x in enumerate(u):
        lib.synth_camera_pose(cp, float(x), p3.ctypes.data_as(ctypes.c_void_p), t3.ctypes.data_as(ctypes.c_void_p))
        pos[i], tan[i] = p3, t3
    return pos, tan


def brick_centres(nbx: int, nby: int, nbz: int, brick: int = 32) -> np.ndarray:
    """Centres (x, y, z) in voxels of a volume's nbx * nby * nbz bricks, in
    brick id order (x fastest)."""
    z, y, x = np.meshgrid(np.arange(nbz), np.arange(nby), np.arange(nbx), indexing="ij")
    return (np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float64) + 0.5) * brick


def frame_requests(nbx: int, nby: int, nbz: int, pos, d0: float, brick: int = 32, max_lod: int = 5):
    """One frame's requests from a camera at pos (voxels) that sees every
    brick: each brick once, at level of detail 0 when its centre lies within
    d0 voxels, else floor(log2(d / d0)) + 1, at most max_lod (one voxel per
    pixel at distance d0, as camera_trace).  Returns (ids u32, lods u8)."""
    d = np.linalg.norm(brick_centres(nbx, nby, nbz, brick) - np.asarray(pos, np.float64), axis=1)
    lod = np.where(d < d0, 0, np.floor(np.log2(np.maximum(d, d0) / d0)) + 1)
    return np.arange(len(d), dtype=np.uint32), np.minimum(lod, max_lod).astype(np.uint8)


def near_bricks(nbx: int, nby: int, nbz: int, pos, radius: float, brick: int = 32) -> np.ndarray:
    """Ids (u32) of the bricks whose centres lie within radius voxels of pos,
    nearest first (ties by id)."""
    d = np.linalg.norm(brick_centres(nbx, nby, nbz, brick) - np.asarray(pos, np.float64), axis=1)
    ids = np.nonzero(d < radius)[0]
    return ids[np.lexsort((ids, d[ids]))].astype(np.uint32)
