"""ctypes binding of libsimlod.so (include/simlod.h): argument marshalling only.

Every step of an insertion runs in the library's HIP kernels; this module
converts Python arguments (torch CUDA tensors, numpy arrays, streams) into the
C ABI's plain pointers and sizes.  There is no fallback: if the shared
library is missing or cannot be loaded, importing this module raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# Always the in-tree build next to this file: tests and the benchmark must
# exercise the product library, never another build of it.
LIB_PATH = os.path.join(_HERE, "libsimlod.so")

OK = 0
ERR_INVALID_ARGUMENT = -1
ERR_OUT_OF_MEMORY = -2
ERR_HIP = -3
ERR_CAPACITY = -4
ERR_POISONED = -5
ERR_KEY_SPACE = -6
ERR_NOT_FOUND = -7
ERR_BUSY = -8

GROUP_GRAPH = 0x1
GROUP_AUTOTUNE = 0x2
MAX_GROUP = 128
TUNE_PASSES = 10

OVF_NODES, OVF_ARENA, OVF_SPILL, OVF_BACKLOG, OVF_WORK, OVF_HASH = 1, 2, 4, 8, 16, 32
OVF_INTERNAL, OVF_HIST = 64, 128

KERNEL_NAMES = ("count", "split", "alloc_points", "sample_store", "alloc_voxels",
                "store_voxels", "finish", "count_hist", "build", "group_batch")

# 16-byte point record: float32 x, y, z and r, g, b, a bytes (rgba as one
# little-endian u32: r in the low byte).
POINT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("rgba", "<u4")])
NODE_DTYPE = np.dtype([("path", "<u8"), ("first", "<u8"), ("count", "<u4"), ("depth", "u1"),
                       ("is_leaf", "u1"), ("reserved", "<u2")])


class Config(ctypes.Structure):
    _fields_ = [
        ("root_min", ctypes.c_float * 3),
        ("root_size", ctypes.c_float),
        ("leaf_capacity", ctypes.c_uint32),
        ("grid_bits", ctypes.c_uint32),
        ("max_depth", ctypes.c_uint32),
        ("chunk_capacity", ctypes.c_uint32),
        ("max_nodes", ctypes.c_uint32),
        ("hist_capacity", ctypes.c_uint32),
        ("arena_bytes", ctypes.c_uint64),
        ("max_batch", ctypes.c_uint64),
        ("spill_capacity", ctypes.c_uint64),
        ("backlog_capacity", ctypes.c_uint64),
        ("device", ctypes.c_int32),
        ("reserved1", ctypes.c_uint32),
        ("arena_ptr", ctypes.c_void_p),
    ]


class SnapshotBuffers(ctypes.Structure):
    _fields_ = [
        ("num_nodes", ctypes.c_uint64),
        ("num_records", ctypes.c_uint64),
        ("num_points", ctypes.c_uint64),
        ("num_voxels", ctypes.c_uint64),
        ("nodes", ctypes.c_void_p),
        ("records", ctypes.c_void_p),
        ("keys", ctypes.c_void_p),
    ]


class StatsData(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "num_nodes", "num_leaves", "num_inner", "num_points", "num_voxels", "chunks_in_use",
        "chunks_pooled", "arena_bytes_used", "arena_bytes_total", "batches", "points_inserted",
        "last_rounds", "last_spilled", "last_new_voxels", "max_rounds", "max_spilled",
        "max_new_voxels", "sum_rounds", "sum_spilled", "sum_new_voxels")] + [("status_bits", ctypes.c_uint32), ("poisoned", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("max_streams", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64), ("max_per_pass", ctypes.c_uint32),
                ("pass_points", ctypes.c_uint32), ("staging_bytes", ctypes.c_uint64)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64 * len(KERNEL_NAMES)),
                ("total_ms", ctypes.c_double * len(KERNEL_NAMES))]


EXPORTS = {
    "simlod_default_config": ([ctypes.POINTER(Config)], ctypes.c_int),
    "simlod_create": ([ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "simlod_insert_batch": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p],
                            ctypes.c_int),
    "simlod_insert_batch_static": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                    ctypes.c_void_p], ctypes.c_int),
    "simlod_snapshot": ([ctypes.c_void_p, ctypes.POINTER(SnapshotBuffers)], ctypes.c_int),
    "simlod_snapshot_subtree": ([ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.POINTER(SnapshotBuffers)], ctypes.c_int),
    "simlod_snapshot_linked": ([ctypes.c_void_p, ctypes.c_uint64,
                                ctypes.POINTER(SnapshotBuffers)], ctypes.c_int),
    "simlod_snapshot_node": ([ctypes.c_void_p, ctypes.c_uint64,
                              ctypes.POINTER(SnapshotBuffers)], ctypes.c_int),
    "simlod_stats": ([ctypes.c_void_p, ctypes.POINTER(StatsData)], ctypes.c_int),
    "simlod_sync": ([ctypes.c_void_p], ctypes.c_int),
    "simlod_reset": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "simlod_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "simlod_set_kernel_timing": ([ctypes.c_void_p, ctypes.c_uint32], ctypes.c_int),
    "simlod_get_kernel_times": ([ctypes.c_void_p, ctypes.POINTER(KernelTimes)], ctypes.c_int),
    "simlod_group_create": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.c_uint32,
                             ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "simlod_group_insert": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                             ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p], ctypes.c_int),
    "simlod_group_shape": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                            ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    "simlod_group_set_kernel_timing": ([ctypes.c_void_p, ctypes.c_uint32], ctypes.c_int),
    "simlod_group_get_kernel_times": ([ctypes.c_void_p, ctypes.POINTER(KernelTimes)],
                                      ctypes.c_int),
    "simlod_group_sync": ([ctypes.c_void_p], ctypes.c_int),
    "simlod_group_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "simlod_tune_chunk_capacity": ([ctypes.POINTER(Config), ctypes.c_void_p, ctypes.c_uint64,
                                    ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "simlod_config_device_bytes": ([ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_uint64)],
                                   ctypes.c_int),
    "simlod_server_create": ([ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)],
                             ctypes.c_int),
    "simlod_server_open": ([ctypes.c_void_p, ctypes.POINTER(Config),
                           ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    "simlod_server_submit": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
                             ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "simlod_server_poll": ([ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "simlod_server_drain": ([ctypes.c_void_p], ctypes.c_int),
    "simlod_server_octree": ([ctypes.c_void_p, ctypes.c_uint32], ctypes.c_void_p),
    "simlod_server_close": ([ctypes.c_void_p, ctypes.c_uint32], ctypes.c_int),
    "simlod_server_wait_closed": ([ctypes.c_void_p], ctypes.c_int),
    "simlod_server_counters": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "simlod_server_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "simlod_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "simlod_last_error": ([], ctypes.c_char_p),
}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
# torch ships its own HIP runtime with the same SONAME (libamdhip64.so.7).
# Loading torch first makes the dynamic linker bind the library to that one
# runtime, so torch's streams and device pointers are valid here; loading the
# library first would put two HIP runtimes into the process.
try:
    import torch  # noqa: F401
except ImportError:  # torch-free use (e.g. host-only checks)
    pass
lib = ctypes.CDLL(LIB_PATH)
for _name, (_args, _res) in EXPORTS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


class SimlodError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})")


def status_string(code: int) -> str:
    return lib.simlod_status_string(code).decode()


def _check(code: int, what: str) -> None:
    if code != OK:
        detail = (lib.simlod_last_error().decode()
                  if code in (ERR_HIP, ERR_OUT_OF_MEMORY, ERR_NOT_FOUND) else "")
        raise SimlodError(code, f"{what} [{detail}]" if detail else what)


def default_config() -> Config:
    cfg = Config()
    _check(lib.simlod_default_config(ctypes.byref(cfg)), "simlod_default_config")
    return cfg


def make_config(root_min=(0.0, 0.0, 0.0), root_size=1.0, leaf_capacity=50_000, grid_bits=7,
                max_depth=16, chunk_capacity=1000, max_nodes=None, arena_bytes=None,
                max_batch=None, spill_capacity=None, backlog_capacity=None, hist_capacity=None,
                device=0) -> Config:
    cfg = default_config()
    cfg.root_min[:] = [float(v) for v in root_min]
    cfg.root_size = float(root_size)
    cfg.leaf_capacity = int(leaf_capacity)
    cfg.grid_bits = int(grid_bits)
    cfg.max_depth = int(max_depth)
    cfg.chunk_capacity = int(chunk_capacity)
    cfg.device = int(device)
    for name, v in (("max_nodes", max_nodes), ("arena_bytes", arena_bytes),
                    ("max_batch", max_batch), ("spill_capacity", spill_capacity),
                    ("backlog_capacity", backlog_capacity), ("hist_capacity", hist_capacity)):
        if v is not None:
            setattr(cfg, name, int(v))
    return cfg


def _stream_ptr(stream) -> int | None:
    if stream is None:
        try:
            import torch

            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream or None
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return stream or None
    return getattr(stream, "cuda_stream", None) or None


def _points_ptr(points):
    """(pointer, count, keepalive) for a torch tensor or numpy array of records."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(points, torch.Tensor):
        if not points.is_contiguous():
            raise ValueError("points tensor must be contiguous")
        nbytes = points.numel() * points.element_size()
        if nbytes % 16:
            raise ValueError("points tensor must hold whole 16-byte records")
        return points.data_ptr(), nbytes // 16, points
    arr = np.ascontiguousarray(points)
    if arr.dtype != POINT_DTYPE:
        if arr.nbytes % 16:
            raise ValueError("points array must hold whole 16-byte records")
        arr = arr.view(np.uint8).reshape(-1)
    return arr.ctypes.data, arr.nbytes // 16, arr


def create(cfg: Config) -> int:
    h = ctypes.c_void_p()
    _check(lib.simlod_create(ctypes.byref(cfg), ctypes.byref(h)), "simlod_create")
    return h.value


def insert_batch(handle: int, points, stream=None) -> None:
    ptr, n, keep = _points_ptr(points)
    _check(lib.simlod_insert_batch(handle, ptr if n else None, n, _stream_ptr(stream)),
           "simlod_insert_batch")
    del keep


def insert_batch_static(handle: int, points, stream=None) -> None:
    """simlod_insert_batch_static: host input staged through the library's
    static device array (no device allocation in the call)."""
    ptr, n, keep = _points_ptr(points)
    _check(lib.simlod_insert_batch_static(handle, ptr if n else None, n, _stream_ptr(stream)),
           "simlod_insert_batch_static")
    del keep


def snapshot(handle: int, path: int | None = None, nodes_only: bool = False,
             linked: bool = False, single: bool = False):
    """Canonical export: (nodes NODE_DTYPE, records POINT_DTYPE, keys uint32)
    of the whole octree, or of the subtree of the node with ``path``; with
    ``nodes_only`` the records and keys come back empty; ``linked`` reads
    the records through the chunk lists; ``single`` exports the node with
    ``path`` alone."""
    if single:
        p = 1 if path is None else path
        call, name = (lambda b: lib.simlod_snapshot_node(handle, p, b)), "simlod_snapshot_node"
    elif linked:
        p = 1 if path is None else path
        call, name = (lambda b: lib.simlod_snapshot_linked(handle, p, b)), "simlod_snapshot_linked"
    elif path is None:
        call, name = (lambda b: lib.simlod_snapshot(handle, b)), "simlod_snapshot"
    else:
        call, name = (lambda b: lib.simlod_snapshot_subtree(handle, path, b)), "simlod_snapshot_subtree"
    s = SnapshotBuffers()
    _check(call(ctypes.byref(s)), name + " (sizes)")
    nodes = np.empty(s.num_nodes, dtype=NODE_DTYPE)
    nrec = 0 if nodes_only else s.num_records
    records = np.empty(nrec, dtype=POINT_DTYPE)
    keys = np.empty(nrec, dtype=np.uint32)
    s.nodes = nodes.ctypes.data
    s.records = None if nodes_only else records.ctypes.data
    s.keys = None if nodes_only else keys.ctypes.data
    _check(call(ctypes.byref(s)), name)
    return nodes[: s.num_nodes], records[:nrec], keys[:nrec]


def stats(handle: int) -> dict:
    st = StatsData()
    _check(lib.simlod_stats(handle, ctypes.byref(st)), "simlod_stats")
    return {name: getattr(st, name) for name, _ in StatsData._fields_}


def sync(handle: int) -> None:
    _check(lib.simlod_sync(handle), "simlod_sync")


def reset(handle: int, stream=None) -> None:
    _check(lib.simlod_reset(handle, _stream_ptr(stream)), "simlod_reset")


def destroy(handle: int) -> None:
    _check(lib.simlod_destroy(handle), "simlod_destroy")


def set_kernel_timing(handle: int, kernels=()) -> None:
    """Times the named kernels (see KERNEL_NAMES); empty disables."""
    if kernels == "all":
        kernels = KERNEL_NAMES
    mask = 0
    for k in kernels:
        mask |= 1 << KERNEL_NAMES.index(k)
    _check(lib.simlod_set_kernel_timing(handle, mask), "simlod_set_kernel_timing")


def get_kernel_times(handle: int) -> dict:
    kt = KernelTimes()
    _check(lib.simlod_get_kernel_times(handle, ctypes.byref(kt)), "simlod_get_kernel_times")
    return {name: (int(kt.launches[i]), float(kt.total_ms[i])) for i, name in enumerate(KERNEL_NAMES)}


@dataclass
class Snapshot:
    nodes: np.ndarray
    records: np.ndarray
    keys: np.ndarray


class Octree:
    """Owning wrapper around one handle."""

    def __init__(self, cfg: Config | None = None, arena=None, **kw):
        """arena: optional caller-owned persistent buffer, a device tensor
        (256-byte aligned); held here until close()."""
        self.cfg = Config.from_buffer_copy(cfg) if cfg is not None else make_config(**kw)
        self._arena = None
        if arena is not None:
            self.cfg.arena_ptr = arena.data_ptr()
            self.cfg.arena_bytes = arena.numel() * arena.element_size()
            self._arena = arena
        self.handle = create(self.cfg)

    def insert(self, points, stream=None) -> None:
        insert_batch(self.handle, points, stream)

    def insert_static(self, points, stream=None) -> None:
        insert_batch_static(self.handle, points, stream)

    def snapshot(self, path: int | None = None, nodes_only: bool = False,
                 linked: bool = False) -> Snapshot:
        return Snapshot(*snapshot(self.handle, path, nodes_only, linked))

    def snapshot_node(self, path: int) -> Snapshot:
        """The node with ``path`` alone (its record and its sorted records)."""
        return Snapshot(*snapshot(self.handle, path, single=True))

    def stats(self) -> dict:
        return stats(self.handle)

    def sync(self) -> None:
        sync(self.handle)

    def reset(self, stream=None) -> None:
        reset(self.handle, stream)

    def close(self) -> None:
        if getattr(self, "handle", None):
            destroy(self.handle)
            self.handle = None
        self._arena = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Batched insertion into several octrees with one pass per call
    (``simlod_group_*``).  The member ``Octree`` objects stay owned by the
    caller and must outlive the group."""

    def __init__(self, trees, graph: bool = False, autotune: bool = False):
        self.trees = list(trees)
        arr = (ctypes.c_void_p * len(self.trees))(*[t.handle for t in self.trees])
        flags = (GROUP_GRAPH if graph else 0) | (GROUP_AUTOTUNE if autotune else 0)
        h = ctypes.c_void_p()
        _check(lib.simlod_group_create(arr, len(self.trees), flags, ctypes.byref(h)),
               "simlod_group_create")
        self.handle = h.value

    def insert(self, batches, stream=None) -> None:
        """batches[i]: device tensor of 16-byte records for member i (may be
        empty or None)."""
        k = len(self.trees)
        ptrs = (ctypes.c_void_p * k)()
        ns = (ctypes.c_uint64 * k)()
        keep = []
        for i, b in enumerate(batches):
            if b is None:
                continue
            p, n, kk = _points_ptr(b)
            ptrs[i] = p if n else None
            ns[i] = n
            keep.append(kk)
        _check(lib.simlod_group_insert(self.handle, ptrs, ns, _stream_ptr(stream)),
               "simlod_group_insert")
        del keep

    def shape(self):
        caps = (ctypes.c_uint32 * 4)()
        state = ctypes.c_uint32()
        _check(lib.simlod_group_shape(self.handle, caps, ctypes.byref(state)), "simlod_group_shape")
        return {"caps": list(caps), "tuned": bool(state.value & 1), "graph": bool(state.value & 2)}

    def set_kernel_timing(self, kernels=()) -> None:
        if kernels == "all":
            kernels = KERNEL_NAMES
        mask = 0
        for k in kernels:
            mask |= 1 << KERNEL_NAMES.index(k)
        _check(lib.simlod_group_set_kernel_timing(self.handle, mask),
               "simlod_group_set_kernel_timing")

    def get_kernel_times(self) -> dict:
        kt = KernelTimes()
        _check(lib.simlod_group_get_kernel_times(self.handle, ctypes.byref(kt)),
               "simlod_group_get_kernel_times")
        return {name: (int(kt.launches[i]), float(kt.total_ms[i]))
                for i, name in enumerate(KERNEL_NAMES)}

    def sync(self) -> None:
        _check(lib.simlod_group_sync(self.handle), "simlod_group_sync")

    def close(self) -> None:
        if self.handle:
            destroy_rc = lib.simlod_group_destroy(self.handle)
            self.handle = None
            _check(destroy_rc, "simlod_group_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_chunk_capacity(cfg: Config, sample, candidates, stream=None):
    """Fastest chunk capacity for inserting ``sample`` (device tensor) into a
    fresh octree of ``cfg``: (best, ms)."""
    p, n, keep = _points_ptr(sample)
    arr = (ctypes.c_uint32 * len(candidates))(*candidates)
    best = ctypes.c_uint32()
    ms = ctypes.c_double()
    _check(lib.simlod_tune_chunk_capacity(ctypes.byref(cfg), p if n else None, n, arr,
                                          len(candidates), _stream_ptr(stream),
                                          ctypes.byref(best), ctypes.byref(ms)),
           "simlod_tune_chunk_capacity")
    del keep
    return int(best.value), float(ms.value)


def config_device_bytes(cfg: Config) -> int:
    b = ctypes.c_uint64()
    _check(lib.simlod_config_device_bytes(ctypes.byref(cfg), ctypes.byref(b)),
           "simlod_config_device_bytes")
    return int(b.value)


class _ServedOctree:
    """Borrowed view of a served stream's octree (owned by the server)."""

    def __init__(self, handle):
        self.handle = handle

    def snapshot(self, path: int | None = None, nodes_only: bool = False) -> Snapshot:
        return Snapshot(*snapshot(self.handle, path, nodes_only))

    def stats(self) -> dict:
        return stats(self.handle)


class Server:
    """Continuous-batching insertion server (``simlod_server_*``)."""

    def __init__(self, max_streams: int, hbm_budget: int, max_per_pass: int = 0, device: int = 0,
                 staging_bytes: int = 0, pass_points: int = 0):
        cfg = ServerConfig(device=device, max_streams=max_streams, hbm_budget=hbm_budget,
                           max_per_pass=max_per_pass, pass_points=pass_points,
                           staging_bytes=staging_bytes)
        h = ctypes.c_void_p()
        _check(lib.simlod_server_create(ctypes.byref(cfg), ctypes.byref(h)), "simlod_server_create")
        self.handle = h.value
        self._keep = {}  # ticket -> the submitted buffer, held until the request is done

    def open(self, cfg: Config):
        """Stream id, or None when the server is busy (no slot or budget)."""
        i = ctypes.c_uint32()
        rc = lib.simlod_server_open(self.handle, ctypes.byref(cfg), ctypes.byref(i))
        if rc == ERR_BUSY:
            return None
        _check(rc, "simlod_server_open")
        return int(i.value)

    def submit(self, sid: int, points) -> int:
        """Queues device tensor or host array ``points`` (host memory needs a
        server created with staging_bytes); the buffer is kept alive here
        until the request is done."""
        p, n, keep = _points_ptr(points)
        t = ctypes.c_uint64()
        _check(lib.simlod_server_submit(self.handle, sid, p if n else None, n, ctypes.byref(t)),
               "simlod_server_submit")
        self._keep[int(t.value)] = keep
        return int(t.value)

    def poll(self, ticket: int):
        """(done, latency_ms, status)."""
        d = ctypes.c_int()
        ms = ctypes.c_double()
        rc = lib.simlod_server_poll(self.handle, ticket, ctypes.byref(d), ctypes.byref(ms))
        if d.value:
            self._keep.pop(ticket, None)
        return bool(d.value), float(ms.value), int(rc)

    def drain(self) -> None:
        _check(lib.simlod_server_drain(self.handle), "simlod_server_drain")
        self._keep.clear()

    def octree(self, sid: int) -> _ServedOctree:
        h = lib.simlod_server_octree(self.handle, sid)
        if not h:
            raise KeyError(sid)
        return _ServedOctree(h)

    def close_stream(self, sid: int) -> None:
        """Closes at once; the octree is destroyed in the background."""
        _check(lib.simlod_server_close(self.handle, sid), "simlod_server_close")

    def wait_closed(self) -> None:
        _check(lib.simlod_server_wait_closed(self.handle), "simlod_server_wait_closed")

    def counters(self) -> dict:
        out = (ctypes.c_uint64 * 4)()
        _check(lib.simlod_server_counters(self.handle, out), "simlod_server_counters")
        return {"passes": out[0], "completed": out[1], "points": out[2], "budget_used": out[3]}

    def close(self) -> None:
        if self.handle:
            rc = lib.simlod_server_destroy(self.handle)
            self.handle = None
            _check(rc, "simlod_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
