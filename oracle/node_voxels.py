"""Voxel lists of single inner nodes from the definition, streamed over the
whole point sequence (``node_voxels.c`` via ctypes).

Test infrastructure only (see the package docstring).  For each listed node
path it keeps, per cell of the node's R^3 grid, the first point in key order
that falls there: the voxel set the definition gives that node if it is inner
(sections "Voxel Sampling Grid" and "Voxel Sampling").  It builds nothing
else, so the voxel lists of the top nodes of clouds far too large for one
oracle octree in a test can be computed in one pass over the points.  The C
code is single-threaded; ctypes releases the GIL during ``feed``, so separate
instances over disjoint node lists can run on separate Python threads.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from .canonical import POINT_DTYPE, LodConfig

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "node_voxels.c")
LIB = os.path.join(_HERE, "liboracle_node_voxels.so")
_lock = threading.Lock()
_lib = None


def compile_library(force: bool = False) -> str:
    """gcc -O2 -ffp-contract=off; returns the path of the shared object."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-Wall", "-Werror", "-o", tmp, SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(compile_library())
            lib.nv_create.restype = ctypes.c_void_p
            lib.nv_create.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_float,
                                      ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32]
            lib.nv_destroy.argtypes = [ctypes.c_void_p]
            lib.nv_feed.restype = ctypes.c_int
            lib.nv_feed.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]
            lib.nv_export.restype = ctypes.c_int64
            lib.nv_export.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.c_void_p]
            _lib = lib
    return _lib


class NodeVoxelOracle:
    """Voxel lists of the nodes ``paths`` (each above max_depth), as if each
    were inner, over the points fed so far."""

    def __init__(self, cfg: LodConfig, paths):
        cfg.validate()
        self.cfg = cfg
        self.paths = [int(p) for p in paths]
        self._lib = _load()
        mn = (ctypes.c_float * 3)(*[float(v) for v in cfg.root_min])
        arr = (ctypes.c_uint64 * max(1, len(self.paths)))(*self.paths)
        self._h = self._lib.nv_create(mn, ctypes.c_float(cfg.root_size), cfg.grid_bits,
                                      cfg.max_depth, arr, len(self.paths))
        if not self._h:
            raise ValueError("node oracle rejected the configuration or a path")

    def close(self):
        if self._h:
            self._lib.nv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def feed(self, points: np.ndarray) -> None:
        """The next points of the sequence, in key order."""
        pts = np.ascontiguousarray(points, dtype=POINT_DTYPE)
        if self._lib.nv_feed(self._h, pts.ctypes.data, len(pts)) != 0:
            raise RuntimeError("node oracle: more than 2^32 - 1 points")

    def voxels(self, path: int):
        """(records POINT_DTYPE, keys uint32) of node ``path``, sorted by key."""
        k = self.paths.index(int(path))
        n = self._lib.nv_export(self._h, k, None, None)
        recs = np.zeros(max(n, 0), dtype=POINT_DTYPE)
        keys = np.zeros(max(n, 0), dtype=np.uint32)
        if n < 0 or self._lib.nv_export(self._h, k, recs.ctypes.data, keys.ctypes.data) != n:
            raise RuntimeError("node oracle export failed")
        return recs, keys


def node_voxels(points: np.ndarray, cfg: LodConfig, paths):
    """{path: (records, keys)} over the whole sequence ``points``."""
    o = NodeVoxelOracle(cfg, paths)
    try:
        o.feed(points)
        return {p: o.voxels(p) for p in o.paths}
    finally:
        o.close()
