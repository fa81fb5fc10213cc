"""Helpers for GPU tests: build library handles matching an oracle config."""

from __future__ import annotations

import sys

import numpy as np

from oracle.canonical import CanonicalTree, LodConfig


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def make_octree(cfg: LodConfig, **caps):
    from paper_2310_03567_amd import simlod

    kw = dict(max_nodes=1 << 16, arena_bytes=512 << 20, max_batch=1 << 20,
              spill_capacity=1 << 20, backlog_capacity=1 << 20)
    kw.update(caps)
    return simlod.Octree(simlod.make_config(
        root_min=cfg.root_min, root_size=cfg.root_size, leaf_capacity=cfg.leaf_capacity,
        grid_bits=cfg.grid_bits, max_depth=cfg.max_depth, chunk_capacity=cfg.chunk_capacity,
        **kw))


def to_device(points: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(points).view(np.uint8).reshape(-1)).to("cuda:0")


def canonical(tree) -> CanonicalTree:
    s = tree.snapshot()
    return CanonicalTree(nodes=s.nodes, records=s.records, keys=s.keys)


def insert_batches(tree, dev_points, sizes) -> None:
    a = 0
    for b in sizes:
        tree.insert(dev_points[a * 16:(a + b) * 16])
        a += b
