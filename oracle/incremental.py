"""O2 wrapper: the sequential C inserter in ``incremental.c`` via ctypes.

Test infrastructure only (see the package docstring).  The shared object is
built by ``__graft_entry__.build()``; if it is missing this module compiles
it with gcc on first use.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from .canonical import NODE_DTYPE, POINT_DTYPE, CanonicalTree, LodConfig, path_depth, subtree

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "incremental.c")
LIB = os.path.join(_HERE, "liboracle_incremental.so")
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
            lib.orc_create.restype = ctypes.c_void_p
            lib.orc_create.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_float,
                                       ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
            lib.orc_destroy.argtypes = [ctypes.c_void_p]
            lib.orc_insert.restype = ctypes.c_int
            lib.orc_insert.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]
            lib.orc_insert_region.restype = ctypes.c_int
            lib.orc_insert_region.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                              ctypes.c_uint64]
            lib.orc_voxels_created_last.restype = ctypes.c_uint64
            lib.orc_voxels_created_last.argtypes = [ctypes.c_void_p]
            lib.orc_sizes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_uint64)]
            lib.orc_export.restype = ctypes.c_int
            lib.orc_export.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
            _lib = lib
    return _lib


class IncrementalOracle:
    """Sequential insertion of batches; ``canonical()`` exports the octree."""

    def __init__(self, cfg: LodConfig):
        cfg.validate()
        self.cfg = cfg
        self._lib = _load()
        mn = (ctypes.c_float * 3)(*[float(v) for v in cfg.root_min])
        self._h = self._lib.orc_create(mn, ctypes.c_float(cfg.root_size), cfg.leaf_capacity,
                                       cfg.grid_bits, cfg.max_depth)
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        self.total = 0
        self.voxels_created_last = 0

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, points: np.ndarray) -> None:
        pts = np.ascontiguousarray(points, dtype=POINT_DTYPE)
        if self._lib.orc_insert(self._h, pts.ctypes.data, len(pts)) != 0:
            raise RuntimeError("oracle insert failed (allocation or key overflow)")
        self.total += len(pts)
        self.voxels_created_last = int(self._lib.orc_voxels_created_last(self._h))

    def insert_region(self, points: np.ndarray, path: int) -> None:
        """Inserts only the points in the region of node ``path``, keeping
        their keys in the whole sequence (see ``orc_insert_region``)."""
        pts = np.ascontiguousarray(points, dtype=POINT_DTYPE)
        rc = self._lib.orc_insert_region(self._h, pts.ctypes.data, len(pts), int(path))
        if rc == -2:
            raise ValueError(f"bad node path {path}")
        if rc != 0:
            raise RuntimeError("oracle insert failed (allocation or key overflow)")
        self.total += len(pts)
        self.voxels_created_last = int(self._lib.orc_voxels_created_last(self._h))

    def region_subtree(self, path: int) -> CanonicalTree:
        """After ``insert_region(.., path)`` calls only: the subtree of node
        ``path`` in canonical form (absolute paths and depths).  If the
        region's points were too few to split the root, that is one leaf
        holding them."""
        t = self.canonical()
        s = subtree(t, path)
        if s is not None:
            return s
        if len(t.nodes) != 1 or not t.nodes["is_leaf"][0]:
            raise RuntimeError("region tree lacks the node although its root split")
        nodes = t.nodes.copy()
        nodes["path"] = path
        nodes["depth"] = path_depth(path)
        return CanonicalTree(nodes=nodes, records=t.records, keys=t.keys)

    def canonical(self) -> CanonicalTree:
        nn = ctypes.c_uint64()
        nr = ctypes.c_uint64()
        self._lib.orc_sizes(self._h, ctypes.byref(nn), ctypes.byref(nr))
        nodes = np.zeros(nn.value, dtype=NODE_DTYPE)
        recs = np.zeros(nr.value, dtype=POINT_DTYPE)
        keys = np.zeros(nr.value, dtype=np.uint32)
        if self._lib.orc_export(self._h, nodes.ctypes.data, recs.ctypes.data, keys.ctypes.data):
            raise RuntimeError("oracle export failed")
        return CanonicalTree(nodes=nodes, records=recs, keys=keys)


def build_incremental(points: np.ndarray, cfg: LodConfig, batch_sizes=None) -> CanonicalTree:
    """Insert ``points`` in consecutive batches (default: one batch)."""
    o = IncrementalOracle(cfg)
    try:
        if batch_sizes is None:
            o.insert(points)
        else:
            a = 0
            for b in batch_sizes:
                o.insert(points[a:a + b])
                a += b
            if a != len(points):
                raise ValueError("batch sizes do not cover the points")
        return o.canonical()
    finally:
        o.close()
