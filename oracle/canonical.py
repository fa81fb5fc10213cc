"""Canonical octree form shared by both oracle implementations.

Test infrastructure only (see the package docstring).

The canonical form is what two octrees built from the same cumulative point
sequence must agree on byte for byte, whatever their memory layout:

* node records in preorder, children visited in octant order 0..7, all eight
  children of an inner node present (a split creates eight children, each
  starting empty -- section "Expanding the Octree");
* a node's path is ``1`` for the root and ``parent_path * 8 + octant`` below
  it (the leading 1 keeps paths of different depths distinct);
* ``count`` is the number of points of a leaf or voxels of an inner node;
* the records of a node are contiguous starting at ``first``; a leaf lists
  its points (records bit-identical to the input) sorted by key, an inner
  node its voxels sorted by the key of the point that chose their colour.

Keys are the 0-based positions of the points in the cumulative insertion
sequence (batch after batch), which equals the order (batch number, index in
batch).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# XYZRGBA, 3 x float32 + 4 x uint8 = 16 bytes: the record format the update
# works on (section "Data Sets", SIM format).  rgba is packed little-endian:
# r in bits 0-7, g in 8-15, b in 16-23, a in 24-31.
POINT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("rgba", "<u4")])

NODE_DTYPE = np.dtype(
    [
        ("path", "<u8"),
        ("first", "<u8"),
        ("count", "<u4"),
        ("depth", "u1"),
        ("is_leaf", "u1"),
        ("reserved", "<u2"),
    ]
)
assert POINT_DTYPE.itemsize == 16 and NODE_DTYPE.itemsize == 24


@dataclass(frozen=True)
class LodConfig:
    """Octree parameters.

    leaf_capacity  T: a leaf splits when it would hold more than T points
                   (section "Octree": 50k; section "Expanding the Octree":
                   "exceeds a given threshold").
    grid_bits      r: inner nodes sample voxels on an R^3 grid, R = 2^r
                   (section "Voxel Sampling Grid": 128^3).
    max_depth      Dmax: nodes at this depth never split (the root is depth 0).
    chunk_capacity C: records per chunk (section "Chunks and the Chunk Pool":
                   1000); it changes the layout, never the canonical form.
    root_min/size  the cubic domain; the paper leaves it open.
    """

    root_min: tuple = (0.0, 0.0, 0.0)
    root_size: float = 1.0
    leaf_capacity: int = 50_000
    grid_bits: int = 7
    max_depth: int = 16
    chunk_capacity: int = 1000

    @property
    def R(self) -> int:
        return 1 << self.grid_bits

    @property
    def K(self) -> int:
        """Bits per axis of the integer point coordinates."""
        return self.max_depth + self.grid_bits

    @property
    def scale(self) -> np.float32:
        """fl32(2^K / root_size), an IEEE single-precision division."""
        return np.float32(2.0**self.K) / np.float32(self.root_size)

    def validate(self) -> None:
        if not (0 <= self.grid_bits <= 8):
            raise ValueError("grid_bits must be in [0, 8]")
        if not (0 <= self.max_depth <= 21):
            raise ValueError("max_depth must be in [0, 21]")
        if self.K > 24:
            raise ValueError("max_depth + grid_bits must be <= 24")
        if self.leaf_capacity < 1 or self.chunk_capacity < 1:
            raise ValueError("capacities must be positive")
        if not (np.float32(self.root_size) > 0 and np.isfinite(np.float32(self.root_size))):
            raise ValueError("root_size must be positive and finite")


@dataclass
class CanonicalTree:
    nodes: np.ndarray  # NODE_DTYPE
    records: np.ndarray  # POINT_DTYPE
    keys: np.ndarray  # uint32
    extra: dict = field(default_factory=dict)

    @property
    def num_points(self) -> int:
        leaf = self.nodes["is_leaf"] == 1
        return int(self.nodes["count"][leaf].sum())

    @property
    def num_voxels(self) -> int:
        inner = self.nodes["is_leaf"] == 0
        return int(self.nodes["count"][inner].sum())

    def node_records(self, i: int):
        n = self.nodes[i]
        a = int(n["first"])
        b = a + int(n["count"])
        return self.records[a:b], self.keys[a:b]

    def by_path(self) -> dict:
        return {int(p): i for i, p in enumerate(self.nodes["path"])}


def path_depth(path: int) -> int:
    """Depth of the node with ``path`` (1 = root, 3 bits per level below)."""
    path = int(path)
    if path < 1 or (path.bit_length() - 1) % 3:
        raise ValueError(f"not a node path: {path}")
    return (path.bit_length() - 1) // 3


def subtree(tree: CanonicalTree, path: int) -> CanonicalTree | None:
    """The subtree rooted at the node with ``path``, in canonical form (paths
    and depths absolute, ``first`` counted from the subtree's first record),
    or None when the tree has no such node.

    In preorder a subtree is the node followed by every later node whose path
    extends it, so it is one contiguous run of nodes and of records.
    """
    d = path_depth(path)
    hit = np.nonzero(tree.nodes["path"] == np.uint64(path))[0]
    if not len(hit):
        return None
    i = int(hit[0])
    depth = tree.nodes["depth"].astype(np.int64)
    # descendants follow directly and are deeper; the run ends at the first
    # node at the subtree root's depth or above
    later = np.nonzero(depth[i + 1:] <= d)[0]
    j = i + 1 + int(later[0]) if len(later) else len(tree.nodes)
    nodes = tree.nodes[i:j].copy()
    a = int(nodes["first"][0])
    b = int(nodes["first"][-1]) + int(nodes["count"][-1])
    nodes["first"] -= np.uint64(a)
    return CanonicalTree(nodes=nodes, records=tree.records[a:b], keys=tree.keys[a:b])


def trees_equal(a: CanonicalTree, b: CanonicalTree) -> bool:
    return (
        a.nodes.shape == b.nodes.shape
        and a.records.shape == b.records.shape
        and a.nodes.tobytes() == b.nodes.tobytes()
        and a.records.tobytes() == b.records.tobytes()
        and np.array_equal(a.keys, b.keys)
    )


def assert_trees_equal(a: CanonicalTree, b: CanonicalTree, what: str = "") -> None:
    """Bit-exact comparison with a readable first difference."""
    pre = f"{what}: " if what else ""
    if a.nodes.shape != b.nodes.shape:
        raise AssertionError(f"{pre}node count {len(a.nodes)} != {len(b.nodes)}")
    for f in NODE_DTYPE.names:
        if f == "reserved":
            continue
        d = np.nonzero(a.nodes[f] != b.nodes[f])[0]
        if len(d):
            i = int(d[0])
            raise AssertionError(
                f"{pre}node {i} field {f}: {a.nodes[i]} != {b.nodes[i]} ({len(d)} nodes differ)"
            )
    if a.records.shape != b.records.shape:
        raise AssertionError(f"{pre}record count {len(a.records)} != {len(b.records)}")
    ka = a.keys.astype(np.uint32)
    kb = b.keys.astype(np.uint32)
    d = np.nonzero(ka != kb)[0]
    if len(d):
        i = int(d[0])
        raise AssertionError(f"{pre}key {i}: {ka[i]} != {kb[i]} ({len(d)} differ)")
    ra = a.records.view(np.uint32).reshape(-1, 4)
    rb = b.records.view(np.uint32).reshape(-1, 4)
    d = np.nonzero((ra != rb).any(axis=1))[0]
    if len(d):
        i = int(d[0])
        raise AssertionError(
            f"{pre}record {i}: {a.records[i]} != {b.records[i]} ({len(d)} differ)"
        )
