"""Loads the hand-worked fixtures under tests/golden."""

from __future__ import annotations

import json
import os

import numpy as np

from oracle.canonical import POINT_DTYPE, LodConfig

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_fig_update():
    with open(os.path.join(GOLDEN, "fig_update_analogue.json")) as f:
        fx = json.load(f)
    c = fx["config"]
    cfg = LodConfig(root_min=tuple(c["root_min"]), root_size=c["root_size"],
                    leaf_capacity=c["leaf_capacity"], grid_bits=c["grid_bits"],
                    max_depth=c["max_depth"], chunk_capacity=c["chunk_capacity"])
    batches = []
    key = 0
    for b in fx["batches"]:
        arr = np.zeros(len(b), dtype=POINT_DTYPE)
        for i, (x, y, z) in enumerate(b):
            arr[i] = (x, y, z, 0xFF000000 + 0x010101 * (key + 1))
            key += 1
        batches.append(arr)
    return cfg, batches, fx["expected"]


def check_against_expected(tree, all_points, expected) -> None:
    """Compares a canonical tree with one hand-derived stage of the fixture."""
    nodes = expected["nodes"]
    assert len(tree.nodes) == len(nodes), f"{len(tree.nodes)} nodes, expected {len(nodes)}"
    for i, e in enumerate(nodes):
        nd = tree.nodes[i]
        assert int(nd["path"]) == e["path"], f"node {i} path"
        assert int(nd["depth"]) == e["depth"], f"node {i} depth"
        assert int(nd["is_leaf"]) == e["is_leaf"], f"node {i} is_leaf"
        recs, keys = tree.node_records(i)
        assert [int(k) for k in keys] == e["keys"], f"node {i} keys {list(keys)} != {e['keys']}"
        for j, k in enumerate(e["keys"]):
            assert recs["rgba"][j] == all_points["rgba"][k], f"node {i} record {j} colour"
            if e["is_leaf"]:
                assert recs[j].tobytes() == all_points[k].tobytes()
            else:
                got = [float(recs[a][j]) for a in "xyz"]
                assert got == e["voxels"][j], f"node {i} voxel {j}: {got} != {e['voxels'][j]}"
