"""O1: the octree LOD written out as its recursive definition (numpy).

Test infrastructure only (see the package docstring).

Build(N, d, P_N) over the cumulative point sequence P, keys = positions in P:

* N is an inner node iff |P_N| > T and d < Dmax (a leaf "spills" when it
  holds more than T points -- section "Expanding the Octree"; Dmax bounds the
  depth).  Its voxels are the occupied cells of the R^3 grid inscribed in N
  (section "Voxel Sampling Grid"), one per cell, placed at the cell centre
  (section "Octree": voxels are points quantized to the cell centre) and
  coloured by the point with the smallest key in that cell (section "Voxel
  Sampling": the first point that projects into an empty cell sets its colour;
  first = smallest key makes this deterministic).  It has 8 children, each
  Build(child_o, d + 1, P_N restricted to octant o), empty ones included.
* Otherwise N is a leaf holding exactly P_N, records bit-identical.

Integer coordinates (the paper leaves the mapping from float positions to
cells open; this is the reading every implementation here follows):

    K     = Dmax + r bits per axis
    scale = fl32(2^K / root_size)
    u     = fl32(fl32(v - root_min) * scale)
    q     = 0 if not (u >= 0)  (negative or NaN)  else min(floor(u), 2^K - 1)

The octant of a point below a node at depth d takes bit K-1-d of each axis
(x in bit 0, y in bit 1, z in bit 2); its cell in a depth-d node is
(q >> (Dmax - d)) & (R - 1) per axis; the global cell coordinate at depth d is
g = q >> (Dmax - d), and the voxel centre is
fl32(root_min + fl32(fl32(g + 0.5) * h_d)) with h_d = root_size * 2^-(r+d).
"""

from __future__ import annotations

import numpy as np

from .canonical import NODE_DTYPE, POINT_DTYPE, CanonicalTree, LodConfig


def quantize(v: np.ndarray, vmin, cfg: LodConfig) -> np.ndarray:
    """Integer coordinate of each value along one axis (uint32)."""
    v = np.asarray(v, dtype=np.float32)
    u = (v - np.float32(vmin)) * cfg.scale  # two float32 roundings
    qmax = np.float32((1 << cfg.K) - 1)
    ok = u >= np.float32(0.0)  # False for NaN and negatives
    q = np.zeros(v.shape, dtype=np.uint32)
    with np.errstate(invalid="ignore"):
        q[ok] = np.minimum(np.floor(u[ok]), qmax).astype(np.uint32)
    return q


def cell_size(cfg: LodConfig, depth: int) -> np.float32:
    """h_d = root_size / (R * 2^d), an exact power-of-two scaling."""
    return np.float32(np.ldexp(np.float32(cfg.root_size), -(cfg.grid_bits + depth)))


def voxel_centre(g: np.ndarray, vmin, cfg: LodConfig, depth: int) -> np.ndarray:
    """Centre of global depth-d cell g along one axis (float32)."""
    h = cell_size(cfg, depth)
    gf = g.astype(np.float32) + np.float32(0.5)  # exact: g < 2^23
    return np.float32(vmin) + gf * h  # product rounded, then sum rounded


def build(points: np.ndarray, cfg: LodConfig, keys: np.ndarray | None = None) -> CanonicalTree:
    """Canonical octree of ``points`` (POINT_DTYPE), the whole sequence so far.

    ``keys`` defaults to 0..n-1 (the points in insertion order).
    """
    cfg.validate()
    points = np.ascontiguousarray(points, dtype=POINT_DTYPE)
    n = len(points)
    if keys is None:
        keys = np.arange(n, dtype=np.uint32)
        order = np.arange(n, dtype=np.int64)
    else:
        keys = np.asarray(keys, dtype=np.uint32)
        if len(np.unique(keys)) != n:
            raise ValueError("keys must be distinct")
        order = np.argsort(keys, kind="stable")

    qx = quantize(points["x"], cfg.root_min[0], cfg)
    qy = quantize(points["y"], cfg.root_min[1], cfg)
    qz = quantize(points["z"], cfg.root_min[2], cfg)

    T, Dmax, R, K = cfg.leaf_capacity, cfg.max_depth, cfg.R, cfg.K
    node_rows: list[tuple] = []
    rec_chunks: list[np.ndarray] = []
    key_chunks: list[np.ndarray] = []
    written = 0

    def visit(idx: np.ndarray, depth: int, path: int) -> None:
        # idx: indices into points, in increasing key order.
        nonlocal written
        m = len(idx)
        if m > T and depth < Dmax:
            shift = Dmax - depth
            gx = qx[idx] >> shift
            gy = qy[idx] >> shift
            gz = qz[idx] >> shift
            mask = np.uint32(R - 1)
            lin = (gx & mask).astype(np.int64) + R * (
                (gy & mask).astype(np.int64) + R * (gz & mask).astype(np.int64)
            )
            # First occurrence in key order = smallest key in the cell.
            _, first = np.unique(lin, return_index=True)
            first = np.sort(first)  # voxel order: by representative key
            reps = idx[first]
            vox = np.empty(len(reps), dtype=POINT_DTYPE)
            vox["x"] = voxel_centre(gx[first], cfg.root_min[0], cfg, depth)
            vox["y"] = voxel_centre(gy[first], cfg.root_min[1], cfg, depth)
            vox["z"] = voxel_centre(gz[first], cfg.root_min[2], cfg, depth)
            vox["rgba"] = points["rgba"][reps]
            node_rows.append((path, written, len(reps), depth, 0, 0))
            rec_chunks.append(vox)
            key_chunks.append(keys[reps])
            written += len(reps)
            b = K - 1 - depth
            octant = (
                ((qx[idx] >> b) & 1)
                | (((qy[idx] >> b) & 1) << 1)
                | (((qz[idx] >> b) & 1) << 2)
            )
            for o in range(8):
                visit(idx[octant == o], depth + 1, path * 8 + o)
        else:
            node_rows.append((path, written, m, depth, 1, 0))
            rec_chunks.append(points[idx])
            key_chunks.append(keys[idx])
            written += m

    visit(order, 0, 1)
    nodes = np.array(node_rows, dtype=NODE_DTYPE)
    records = (
        np.concatenate(rec_chunks) if rec_chunks else np.empty(0, dtype=POINT_DTYPE)
    ).astype(POINT_DTYPE, copy=False)
    allkeys = np.concatenate(key_chunks).astype(np.uint32) if key_chunks else np.empty(0, np.uint32)
    return CanonicalTree(nodes=nodes, records=records, keys=allkeys)
