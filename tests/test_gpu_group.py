"""Batched insertion (simlod_group_*): several octrees, one pass per call.

Each member's canonical octree must equal the oracle's for that member's
own cumulative point sequence, bit for bit, whatever the mix of members,
batch sizes, launch shapes (autotuning) and graph replay.
"""

from __future__ import annotations

import numpy as np
import pytest

from oracle import POINT_DTYPE, LodConfig, assert_trees_equal
from oracle import definition as O1
from tests.gpu_util import canonical, log, make_octree, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_03567_amd import simlod  # noqa: F401  (fails loudly if not built)


def _cloud(rng, n):
    xyz = rng.random((n, 3)) ** rng.choice([1, 2, 4])
    p = np.zeros(n, dtype=POINT_DTYPE)
    p["x"], p["y"], p["z"] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    p["rgba"] = rng.integers(0, 2**32, n, dtype=np.uint32)
    return p


def _members(rng, k):
    """k different configurations and clouds of uneven size."""
    out = []
    for i in range(k):
        cfg = LodConfig(leaf_capacity=int(rng.choice([3, 20, 200, 2000])),
                        grid_bits=int(rng.integers(1, 6)), max_depth=int(rng.integers(3, 12)),
                        chunk_capacity=int(rng.choice([1, 7, 100, 1000])))
        n = int(np.exp(rng.uniform(np.log(10), np.log(60_000))))
        out.append((cfg, _cloud(rng, n)))
    return out


def _run(members, passes, graph, autotune, seed, max_batch=None):
    from paper_2310_03567_amd import simlod

    rng = np.random.default_rng(seed)
    trees = [make_octree(cfg, max_nodes=1 << 15, arena_bytes=256 << 20,
                         **({"max_batch": max_batch} if max_batch else {}))
             for cfg, _ in members]
    devs = [to_device(p) for _, p in members]
    # uneven cuts per member, some empty
    cuts = []
    for _, p in members:
        c = np.sort(rng.integers(0, len(p) + 1, passes - 1))
        cuts.append(np.concatenate([[0], c, [len(p)]]))
    with simlod.Group(trees, graph=graph, autotune=autotune) as g:
        for k in range(passes):
            g.insert([d[int(c[k]) * 16:int(c[k + 1]) * 16] for d, c in zip(devs, cuts)])
            if k % 3 == 1:  # eager work and a sync between replays
                trees[0].stats()
        g.sync()
        shape = g.shape()
    got = [canonical(t) for t in trees]
    stats = [t.stats() for t in trees]
    for t in trees:
        t.close()
    return got, stats, shape


@pytest.mark.parametrize("graph,autotune", [(False, False), (True, False), (True, True)])
def test_group_members_equal_their_own_oracle(graph, autotune):
    from paper_2310_03567_amd import simlod

    rng = np.random.default_rng(21)
    members = _members(rng, 12)
    passes = simlod.TUNE_PASSES + 4 if autotune else 6
    log(f"case: group of 12, {passes} passes, graph={graph} autotune={autotune}")
    got, stats, shape = _run(members, passes, graph, autotune, seed=22)
    for i, ((cfg, p), t, st) in enumerate(zip(members, got, stats)):
        assert st["status_bits"] == 0
        assert_trees_equal(t, O1.build(p, cfg), f"member {i} n={len(p)}")
    if autotune:
        assert shape["tuned"] and all(c in (256, 512, 1024, 2048, 4096) for c in shape["caps"])
    if graph:
        assert shape["graph"]


def test_group_cuts_batches_above_max_batch():
    rng = np.random.default_rng(23)
    members = _members(rng, 5)
    log("case: group, max_batch 5000")
    got, _, _ = _run(members, 3, graph=True, autotune=False, seed=24, max_batch=5_000)
    for i, ((cfg, p), t) in enumerate(zip(members, got)):
        assert_trees_equal(t, O1.build(p, cfg), f"member {i}")


def test_group_of_one_equals_single_insertion():
    import pointgen

    p = pointgen.tiny_planes(300_000, seed=25)
    cfg = LodConfig(leaf_capacity=4_000, grid_bits=6, max_depth=10, chunk_capacity=333)
    log("case: group of one vs single insertion")
    got, _, _ = _run([(cfg, p)], 4, graph=True, autotune=False, seed=26)
    assert_trees_equal(got[0], O1.build(p, cfg))


def test_member_overflow_poisons_only_that_member():
    from paper_2310_03567_amd import simlod

    rng = np.random.default_rng(27)
    ok_cfg = LodConfig(leaf_capacity=50, grid_bits=3, max_depth=8)
    a, b = _cloud(rng, 20_000), _cloud(rng, 20_000)
    log("case: group member overflow")
    small = make_octree(ok_cfg, max_nodes=17)  # overflows its node table
    good = make_octree(ok_cfg, max_nodes=1 << 14)
    with simlod.Group([small, good]) as g:
        g.insert([to_device(a), to_device(b)])
        with pytest.raises(simlod.SimlodError) as e:
            g.sync()
        assert e.value.code == simlod.ERR_CAPACITY
        with pytest.raises(simlod.SimlodError) as e:
            g.insert([None, to_device(b[:0])])
        assert e.value.code == simlod.ERR_POISONED
    assert small.stats()["status_bits"] != 0
    assert_trees_equal(canonical(good), O1.build(b, ok_cfg))
    small.close()
    good.close()


def test_chunk_capacity_tuner_picks_a_candidate():
    import pointgen
    from paper_2310_03567_amd import simlod

    p = pointgen.tiny_planes(200_000, seed=28)
    cfg = simlod.make_config(leaf_capacity=5_000, grid_bits=6, max_depth=10,
                             max_nodes=1 << 15, arena_bytes=512 << 20, max_batch=1 << 20,
                             spill_capacity=1 << 20, backlog_capacity=1 << 20)
    log("case: chunk tuner")
    best, ms = simlod.tune_chunk_capacity(cfg, to_device(p), [250, 1000, 4000])
    assert best in (250, 1000, 4000) and ms > 0


def test_captured_group_of_one_takes_the_grouped_order():
    """A group of one whose capacity is a large pass (5M points) replays,
    from a graph, the pass that copies the batch into the leaf-grouped
    order; passes of uneven size (one below the large-pass size) must give
    the sequential oracle's octree."""
    import pointgen
    from oracle.incremental import IncrementalOracle
    from paper_2310_03567_amd import simlod

    p = pointgen.dense_scan(9_000_000, seed=27)
    cfg = LodConfig(root_size=64.0, leaf_capacity=20_000, grid_bits=6, max_depth=12,
                    chunk_capacity=500)
    dev = to_device(p)
    cuts = [0, 1_500_000, 6_000_000, 9_000_000]
    tree = make_octree(cfg, arena_bytes=4 << 30, max_batch=5_000_000, spill_capacity=8 << 20,
                       backlog_capacity=8 << 20, max_nodes=1 << 18)
    log("case: captured group of one, 5M capacity, passes of 1.5M, 4.5M, 3M")
    with simlod.Group([tree], graph=True) as g:
        for a, b in zip(cuts[:-1], cuts[1:]):
            g.insert([dev[a * 16:b * 16]])
        g.sync()
        assert g.shape()["graph"]
    o = IncrementalOracle(cfg)
    for a, b in zip(cuts[:-1], cuts[1:]):
        o.insert(p[a:b])
    st = tree.stats()
    assert st["status_bits"] == 0 and st["num_points"] == len(p)
    assert_trees_equal(canonical(tree), o.canonical(), "captured group of one")
    o.close()
    tree.close()
