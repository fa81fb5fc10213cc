"""Pins of the streamed single-node voxel oracle (oracle/node_voxels.c).

* Against O1, the recursive definition (independent code): for every inner
  node of O1's octree, the node oracle's voxel records and keys are identical,
  with the points fed in several pieces (keys continue across calls).
* Closed forms: a 1-cell grid gives one voxel per node at its exact centre,
  coloured by the smallest key of its region; an empty region gives none; the
  lattice case gives, at the root, the smallest key among each cell's 8 points.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

from oracle import POINT_DTYPE, LodConfig
from oracle import definition as O1
from oracle.node_voxels import NodeVoxelOracle, node_voxels


def _points(xyz, rgba):
    xyz = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    p = np.zeros(len(xyz), dtype=POINT_DTYPE)
    p["x"], p["y"], p["z"] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    p["rgba"] = rgba
    return p


@pytest.mark.parametrize("seed,T,r,dmax,n,mn,size", [
    (0, 5, 2, 5, 800, 0.0, 1.0),
    (1, 20, 3, 6, 3000, -1.3, 3.7),
    (2, 1, 1, 4, 300, 0.0, 1.0),
    (3, 50, 4, 8, 6000, 100.25, 1000.0),
    (4, 7, 0, 5, 500, 0.0, 1.0),
])
def test_node_voxels_equal_definition_on_every_inner_node(seed, T, r, dmax, n, mn, size):
    rng = np.random.default_rng(seed)
    cfg = LodConfig(leaf_capacity=T, grid_bits=r, max_depth=dmax, root_min=(mn, mn, mn),
                    root_size=size)
    u = rng.random((n, 3)) ** 3  # clustered toward a corner: several depths
    if seed == 2:
        u[::17] = [np.nan, -2.0, 5.0]  # out-of-domain and NaN coordinates clamp
    p = _points(np.float32(mn) + u * size, rng.integers(0, 2**32, n, dtype=np.uint32))
    tree = O1.build(p, cfg)
    inner = [i for i in range(len(tree.nodes)) if not tree.nodes["is_leaf"][i]]
    assert inner, "the case must have inner nodes"
    paths = [int(tree.nodes["path"][i]) for i in inner]
    o = NodeVoxelOracle(cfg, paths)
    for a in range(0, n, 333):  # streamed in pieces
        o.feed(p[a:a + 333])
    for i, path in zip(inner, paths):
        want_r, want_k = tree.node_records(i)
        got_r, got_k = o.voxels(path)
        assert got_k.tolist() == want_k.tolist(), f"keys of node {path}"
        assert got_r.tobytes() == want_r.tobytes(), f"records of node {path}"
    o.close()


def _node_box(path):
    octs = []
    while path > 1:
        octs.append(path & 7)
        path >>= 3
    octs.reverse()
    lo = [Fraction(0)] * 3
    size = Fraction(1)
    for o in octs:
        size /= 2
        lo = [lo[a] + size * ((o >> a) & 1) for a in range(3)]
    return octs, lo, size


def test_single_cell_grid_gives_node_centres_and_region_minimum():
    cfg = LodConfig(leaf_capacity=4, grid_bits=0, max_depth=6)
    rng = np.random.default_rng(7)
    xyz = rng.random((500, 3)) * 0.5  # nothing in the upper half of any axis
    p = _points(xyz, rng.integers(0, 2**32, 500, dtype=np.uint32))
    paths = [1, 8, 9, 15, 64, 65, 71]  # 15 = octant 7 of the root: empty region
    vox = node_voxels(p, cfg, paths)
    q = [O1.quantize(p[a], 0.0, cfg) for a in "xyz"]
    for path in paths:
        octs, lo, size = _node_box(path)
        sel = np.ones(len(p), bool)
        for d, o in enumerate(octs):
            for a in range(3):
                sel &= ((q[a] >> (cfg.K - 1 - d)) & 1) == ((o >> a) & 1)
        recs, keys = vox[path]
        if not sel.any():
            assert len(keys) == 0, path
            continue
        k = int(np.nonzero(sel)[0].min())
        assert keys.tolist() == [k]
        assert [Fraction(float(recs[0][a])) for a in "xyz"] == [lo[a] + size / 2 for a in range(3)]
        assert int(recs[0]["rgba"]) == int(p[k]["rgba"])


def test_lattice_root_takes_the_smallest_key_of_each_cell():
    cfg = LodConfig(leaf_capacity=7, grid_bits=2, max_depth=2)
    idx = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"),
                   -1).reshape(-1, 3)
    rng = np.random.default_rng(4)
    perm = rng.permutation(len(idx))
    p = _points((idx[perm] + 0.5) / 8.0, rng.integers(0, 2**32, len(idx), dtype=np.uint32))
    recs, keys = node_voxels(p, cfg, [1])[1]
    cell = idx[perm] // 2
    lin = cell[:, 0] + 4 * (cell[:, 1] + 4 * cell[:, 2])
    assert keys.tolist() == sorted(int(np.nonzero(lin == c)[0].min()) for c in range(64))
    # each root voxel at its cell's centre: (2c + 1) / 8
    for r_, k in zip(recs, keys):
        c = cell[k]
        assert [float(r_[a]) for a in "xyz"] == [(2 * c[a] + 1) / 8.0 for a in range(3)]


def test_rejects_paths_that_are_not_nodes_above_max_depth():
    cfg = LodConfig(leaf_capacity=4, grid_bits=1, max_depth=2)
    for bad in ([0], [2 ** 3 + 9], [1 * 64 + 3]):  # 0, not a path, depth 2 = Dmax
        with pytest.raises(ValueError):
            NodeVoxelOracle(cfg, bad)
