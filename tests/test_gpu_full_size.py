"""Parity at the full sizes of the benchmark workloads, in the launch
configuration ``bench.py`` times (same capacities, same batch cut).

* aerial (100M points, 1M-point batches): the whole canonical octree equals
  the sequential oracle's, bit for bit.
* dense scan (1B points, 10M-point batches): too large for one oracle run
  inside a test, so (i) the whole node table is checked against what the
  definition fixes at any size (topology from region point totals, voxel
  counts, chunk totals), and (ii) sampled subtrees are compared bit for bit
  with the oracle fed only each subtree's region (keys of the whole sequence
  kept), which by the recursive definition is exactly that subtree.
"""

from __future__ import annotations

import time

import numpy as np
import pytest

from oracle import LodConfig, assert_trees_equal
from oracle.incremental import IncrementalOracle
from tests.gpu_util import log, to_device

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_03567_amd import simlod  # noqa: F401  (fails loudly if not built)


def _canonical(s):
    from oracle.canonical import CanonicalTree

    return CanonicalTree(nodes=s.nodes, records=s.records, keys=s.keys)


def _build_on_gpu(name, pts):
    import torch

    import bench
    from paper_2310_03567_amd import simlod

    B = bench.WORKLOADS[name]["batch"]
    dev = to_device(pts)
    tree = simlod.Octree(bench.octree_config(name))
    t0 = time.perf_counter()
    for i in range(0, len(pts), B):
        tree.insert(dev[i * 16:(i + B) * 16])
    tree.sync()
    log(f"{name}: {len(pts)} points inserted in {time.perf_counter() - t0:.2f} s")
    del dev
    torch.cuda.empty_cache()
    return tree


def _oracle_config(name):
    import bench

    w = bench.WORKLOADS[name]
    return LodConfig(root_min=w["root_min"], root_size=w["root_size"])


@pytest.mark.timeout(900)
def test_aerial_100M_whole_octree_equals_sequential_oracle():
    import bench

    log("case: aerial 100M, 1M-point batches, whole octree")
    t0 = time.perf_counter()
    pts = bench.generate("aerial")
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    tree = _build_on_gpu("aerial", pts)
    st = tree.stats()
    assert st["status_bits"] == 0 and st["num_points"] == len(pts)
    got = _canonical(tree.snapshot())
    tree.close()
    log(f"gpu snapshot: {len(got.nodes)} nodes, {len(got.records)} records")
    cfg = _oracle_config("aerial")
    o = IncrementalOracle(cfg)
    B = bench.WORKLOADS["aerial"]["batch"]
    t0 = time.perf_counter()
    for i in range(0, len(pts), B):
        o.insert(pts[i:i + B])
    log(f"oracle: {time.perf_counter() - t0:.1f} s")
    want = o.canonical()
    o.close()
    assert_trees_equal(got, want, "aerial 100M")


def _check_node_table(nodes, total, cfg: LodConfig, chunks_in_use: int):
    """What the definition fixes about the node table at any size."""
    T, Dmax, R, C = cfg.leaf_capacity, cfg.max_depth, cfg.R, cfg.chunk_capacity
    path = nodes["path"].astype(np.int64)
    depth = nodes["depth"].astype(np.int64)
    leaf = nodes["is_leaf"] == 1
    count = nodes["count"].astype(np.int64)
    assert path[0] == 1 and depth[0] == 0
    index = {int(p): i for i, p in enumerate(path)}
    assert len(index) == len(nodes)
    # region point totals, children before parents in reverse preorder
    region = np.where(leaf, count, 0)
    for i in range(len(nodes) - 1, -1, -1):
        if leaf[i]:
            continue
        kids = [index.get(int(path[i]) * 8 + o) for o in range(8)]
        assert None not in kids, f"inner node {path[i]} lacks a child"
        assert all(depth[k] == depth[i] + 1 for k in kids)
        region[i] = sum(region[k] for k in kids)
    # every node other than the root is a child of an inner node
    parents = path[1:] >> 3
    assert all(not leaf[index[int(q)]] for q in np.unique(parents))
    assert region[0] == total
    inner = ~leaf
    assert (region[inner] > T).all() and (depth[inner] < Dmax).all()
    assert (region[leaf & (depth < Dmax)] <= T).all()
    assert (count[inner] >= 1).all() and (count[inner] <= np.minimum(region[inner], R ** 3)).all()
    assert int(((count + C - 1) // C).sum()) == chunks_in_use


@pytest.mark.timeout(1200)
def test_dense_scan_1B_node_table_and_sampled_subtrees():
    import bench

    log("case: dense scan 1B, 10M-point batches")
    t0 = time.perf_counter()
    pts = bench.generate("dense")
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    tree = _build_on_gpu("dense", pts)
    cfg = _oracle_config("dense")
    st = tree.stats()
    assert st["status_bits"] == 0 and st["num_points"] == len(pts)
    nodes = tree.snapshot(nodes_only=True).nodes
    log(f"node table: {len(nodes)} nodes, depth {int(nodes['depth'].max())}, "
        f"{st['num_voxels']} voxels")
    _check_node_table(nodes, len(pts), cfg, st["chunks_in_use"])

    # sampled subtrees: a depth-1 octant (the smallest inner one), the
    # depth-3 ancestor of the deepest node, and the most populated leaf
    path = nodes["path"].astype(np.int64)
    depth = nodes["depth"].astype(np.int64)
    leaf = nodes["is_leaf"] == 1
    d1 = np.nonzero((depth == 1) & ~leaf)[0]
    pts_below = {}
    for i in d1:
        sub = tree.snapshot(int(path[i]), nodes_only=True).nodes
        pts_below[int(path[i])] = int(sub["count"][sub["is_leaf"] == 1].sum())
    octant = min(pts_below, key=pts_below.get)
    deep = int(path[np.argmax(depth)])
    deep3 = deep >> (3 * (int(depth.max()) - 3))
    big_leaf = int(path[leaf][np.argmax(nodes["count"][leaf])])
    B = bench.WORKLOADS["dense"]["batch"]
    for p in (deep3, big_leaf, octant):
        log(f"subtree {p} (depth {(p.bit_length() - 1) // 3})")
        t0 = time.perf_counter()
        got = _canonical(tree.snapshot(p))
        o = IncrementalOracle(cfg)
        for i in range(0, len(pts), B):
            o.insert_region(pts[i:i + B], p)
        want = o.region_subtree(p)
        o.close()
        log(f"  {len(got.nodes)} nodes, {len(got.records)} records, "
            f"{time.perf_counter() - t0:.1f} s")
        assert_trees_equal(got, want, f"dense subtree {p}")
    tree.close()
