"""Seeded synthetic point clouds for tests and benchmarks.

Input generators only: this module computes no part of the octree and is
shared by the HIP path's tests/benchmarks and the oracle as the one common
source of inputs.  All records are 16-byte XYZRGBA (float32 x, y, z; rgba
bytes packed little-endian into a u32).

Workloads (the paper's data sets are not available; these stand in for their
shapes, matching sizes in order of magnitude only):

* ``tiny_planes`` -- 1M points, 95% uniform on 3 random axis-aligned planes
  inside the unit cube, 5% uniform volume noise, random rgba; 10 batches of
  100k in generation order (seed 0).
* ``aerial`` -- 100M points on a 1 km x 1 km heightfield (8-octave fBm value
  noise, 100 m relief) whose density varies 4x with a low-frequency mask,
  colour from height; batches of 1M cut from Morton order and shuffled
  (seed 1).  Stands in for aerial LiDAR (the paper's Morro Bay and the
  outskirts of Retz).
* ``dense_scan`` -- 1B points on the 2,000 primitives (slabs, walls, furniture
  boxes) of a synthetic 60 x 60 x 15 m building in a 64 m cube, with 200
  Gaussian hotspots (sigma 0.5 m, 20x peak density), colour per primitive
  plus jitter, in scan-like primitive-by-primitive order; batches of 10M
  (seed 2).  Stands in for the terrestrial and photogrammetry scans
  (Endeavor, Chiller, Meroe, the town centre of Retz).
* ``cloud_set`` -- 64 independent clouds, sizes log-uniform in 100k..50M,
  each an aerial heightfield or a dense building scan chosen by the seed
  (seed 3); each is cut into 10 batches and step s inserts batch s of every
  cloud.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

POINT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("rgba", "<u4")])

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pointgen.c")
_LIB = os.path.join(_HERE, "libpointgen.so")
_lock = threading.Lock()
_lib = None

ORDERS = {"generation": 0, "morton": 1, "morton_shuffled": 2, "random": 3}


def compile_library(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(compile_library())
            lib.pg_aerial.restype = ctypes.c_int
            lib.pg_aerial.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_float), ctypes.c_float, ctypes.c_int]
            lib.pg_dense_scan.restype = ctypes.c_int
            lib.pg_dense_scan.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_int]
            _lib = lib
    return _lib


def _threads() -> int:
    n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, min(n, 16))


def tiny_planes(n: int = 1_000_000, seed: int = 0) -> np.ndarray:
    """Points on 3 random axis-aligned planes in [0,1)^3 plus 5% volume noise."""
    rng = np.random.default_rng(seed)
    axes = rng.integers(0, 3, 3)
    offsets = rng.random(3)
    u = rng.random((n, 3))
    on_plane = rng.random(n) < 0.95
    which = rng.integers(0, 3, n)
    xyz = u.copy()
    for k in range(3):
        sel = on_plane & (which == k)
        xyz[sel, axes[k]] = offsets[k]
    p = np.empty(n, dtype=POINT_DTYPE)
    xyz32 = xyz.astype(np.float32)
    xyz32 = np.minimum(xyz32, np.float32(np.nextafter(np.float32(1), np.float32(0))))
    p["x"], p["y"], p["z"] = xyz32[:, 0], xyz32[:, 1], xyz32[:, 2]
    p["rgba"] = rng.integers(0, 2**32, n, dtype=np.uint32)
    return p


def aerial(n: int = 100_000_000, seed: int = 1, order: str = "morton_shuffled",
           batch: int = 1_000_000, extent: float = 1000.0, z0: float = 200.0,
           relief: float = 100.0, cube_min=(0.0, 0.0, 0.0), cube_size: float = 1024.0,
           threads: int | None = None) -> np.ndarray:
    """Aerial-LiDAR-shaped heightfield cloud (see pointgen.c)."""
    out = np.empty(n, dtype=POINT_DTYPE)
    mn = (ctypes.c_float * 3)(*[float(v) for v in cube_min])
    rc = _load().pg_aerial(out.ctypes.data, n, seed, extent, z0, relief, ORDERS[order], batch,
                           mn, cube_size, threads or _threads())
    if rc != 0:
        raise RuntimeError(f"pg_aerial failed ({rc})")
    return out


def dense_scan(n: int = 1_000_000_000, seed: int = 2, threads: int | None = None) -> np.ndarray:
    """Dense-scan-shaped building cloud in scan-like order (see pointgen.c).

    The root cube is [0, 64)^3."""
    out = np.empty(n, dtype=POINT_DTYPE)
    rc = _load().pg_dense_scan(out.ctypes.data, n, seed, threads or _threads())
    if rc != 0:
        raise RuntimeError(f"pg_dense_scan failed ({rc})")
    return out


AERIAL_CUBE = ((0.0, 0.0, 0.0), 1024.0)
DENSE_CUBE = ((0.0, 0.0, 0.0), 64.0)


def cloud_set(count: int = 64, seed: int = 3, lo: float = 1e5, hi: float = 5e7,
              scale: float = 1.0):
    """Independent clouds of uneven size for batched insertion: sizes
    log-uniform in [lo, hi] (times ``scale``), each one an aerial
    heightfield or a dense building scan chosen by the seed.

    Returns a list of dicts: kind, points, root_min, root_size, seed."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), count)) * scale
    kinds = rng.integers(0, 2, count)
    out = []
    for i in range(count):
        n = max(1, int(sizes[i]))
        s = seed * 1000 + i
        if kinds[i] == 0:
            pts = aerial(n, seed=s, order="morton_shuffled", batch=max(1, n // 10))
            mn, size = AERIAL_CUBE
            kind = "aerial"
        else:
            pts = dense_scan(n, seed=s)
            mn, size = DENSE_CUBE
            kind = "dense"
        out.append(dict(kind=kind, points=pts, root_min=mn, root_size=size, seed=s))
    return out


def batches(points: np.ndarray, size: int):
    """Consecutive batch slices of ``size`` points (last one ragged)."""
    return [points[i:i + size] for i in range(0, len(points), size)]
