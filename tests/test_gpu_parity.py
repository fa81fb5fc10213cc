"""Bit-exact parity of the HIP insertion path with the CPU oracle.

Every test inserts seeded synthetic points through the C ABI (via the ctypes
binding) and compares the canonical snapshot with the oracle element by
element: node records, point/voxel records and keys must be identical.
"""

from __future__ import annotations

import numpy as np
import pytest

from oracle import POINT_DTYPE, LodConfig, assert_trees_equal
from oracle import definition as O1
from oracle.incremental import IncrementalOracle
from tests.golden_util import check_against_expected, load_fig_update
from tests.gpu_util import canonical, insert_batches, log, make_octree, to_device
from tests.invariants import check_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_03567_amd import simlod  # noqa: F401  (fails loudly if not built)


def _pts(xyz, rgba):
    xyz = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    p = np.zeros(len(xyz), dtype=POINT_DTYPE)
    p["x"], p["y"], p["z"] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    p["rgba"] = rgba
    return p


def test_hand_worked_example():
    cfg, batches, expected = load_fig_update()
    log("case: fig-update analogue T=5 C=2")
    with make_octree(cfg) as tree:
        seen = []
        for b, e in zip(batches, expected):
            seen.append(b)
            tree.insert(to_device(b))
            got = canonical(tree)
            allp = np.concatenate(seen)
            check_against_expected(got, allp, e)
            st = tree.stats()
            assert st["chunks_in_use"] == e["chunks"]
            assert st["status_bits"] == 0


def _tiny(rng, n):
    mode = rng.integers(0, 4)
    if mode == 0:
        xyz = rng.random((n, 3))
    elif mode == 1:
        xyz = rng.integers(0, 8, (n, 3)) / 8.0
    elif mode == 2:
        xyz = rng.random((n, 3)) ** 4
    else:
        xyz = np.repeat(rng.random((n // 10 + 1, 3)), 10, axis=0)[:n]
    if n and rng.random() < 0.3:
        xyz[rng.integers(0, n)] = [np.nan, -3.0, 7.0]
        xyz[rng.integers(0, n)] = [np.inf, 0.5, -np.inf]
    return _pts(xyz, rng.integers(0, 2**32, n, dtype=np.uint32))


def test_many_tiny_configurations():
    rng = np.random.default_rng(11)
    cases = 0
    for T in (1, 2, 5, 17):
        for r in (0, 1, 2, 3):
            for dmax in (0, 1, 3, 6):
                C = int(rng.choice([1, 2, 3, 7, 1000]))
                cfg = LodConfig(leaf_capacity=T, grid_bits=r, max_depth=dmax, chunk_capacity=C)
                n = int(rng.integers(0, 300))
                p = _tiny(rng, n)
                parts = np.diff(np.unique(np.concatenate([[0, n], rng.integers(0, n + 1, 4)])))
                log(f"case: tiny T={T} r={r} Dmax={dmax} C={C} n={n} parts={parts.tolist()}")
                with make_octree(cfg, max_nodes=1 << 14, arena_bytes=64 << 20) as tree:
                    insert_batches(tree, to_device(p), parts.tolist())
                    got = canonical(tree)
                    st = tree.stats()
                assert_trees_equal(got, O1.build(p, cfg), f"T={T} r={r} Dmax={dmax} C={C} n={n}")
                assert st["status_bits"] == 0
                assert st["chunks_in_use"] == sum(-(-int(c) // C) for c in got.nodes["count"])
                cases += 1
    assert cases == 64


def test_every_batch_matches_sequential_oracle_on_planes():
    """Plain method, tiny workload shape (1M points on 3 planes + 5% noise,
    10 batches of 100k, T = 50k, 128^3 grid, Dmax 16): snapshot after every
    batch equals the sequential oracle's octree after the same batches."""
    import pointgen

    p = pointgen.tiny_planes(1_000_000, seed=0)
    cfg = LodConfig()
    dev = to_device(p)
    o = IncrementalOracle(cfg)
    with make_octree(cfg, arena_bytes=2 << 30) as tree:
        for k in range(10):
            log(f"case: planes batch {k}")
            b = slice(k * 100_000, (k + 1) * 100_000)
            tree.insert(dev[b.start * 16:b.stop * 16])
            o.insert(p[b])
            assert_trees_equal(canonical(tree), o.canonical(), f"after batch {k}")
        st = tree.stats()
    assert st["num_points"] == 1_000_000 and st["status_bits"] == 0
    assert st["num_inner"] >= 1


def test_large_passes_with_the_candidate_table_match_sequential_oracle():
    """Passes of 4.5M points take the kernels' large-pass shape (the LDS
    candidate table for voxel claims, the widened histogram round); small
    passes do not.  Two such passes of a scan-ordered dense cloud (points of
    a strip in random order, so tiles overflow the candidate table) against
    the sequential oracle, after each pass."""
    import pointgen

    p = pointgen.dense_scan(9_000_000, seed=5)
    cfg = LodConfig(root_size=64.0, leaf_capacity=20_000, grid_bits=6, max_depth=12,
                    chunk_capacity=500)
    dev = to_device(p)
    o = IncrementalOracle(cfg)
    with make_octree(cfg, arena_bytes=4 << 30, max_batch=5_000_000, spill_capacity=8 << 20,
                     backlog_capacity=8 << 20, max_nodes=1 << 18) as tree:
        for k in range(2):
            log(f"case: large pass {k}, 4.5M dense-scan points")
            b = slice(k * 4_500_000, (k + 1) * 4_500_000)
            tree.insert(dev[b.start * 16:b.stop * 16])
            o.insert(p[b])
            assert_trees_equal(canonical(tree), o.canonical(), f"after large pass {k}")
        st = tree.stats()
    o.close()
    assert st["status_bits"] == 0 and st["num_inner"] > 1 and st["max_spilled"] > 0


@pytest.mark.parametrize("T,r,dmax,C", [(17, 2, 6, 1), (1, 0, 3, 7), (5000, 3, 9, 1000)])
def test_grouped_passes_of_random_clouds(T, r, dmax, C):
    """Passes of 4.5M points take the leaf-grouped order; uniformly random
    points (nearly every point of a window in another leaf), repeated points,
    NaN/inf and out-of-domain points, in small-T / small-grid / C = 1
    configurations: two passes against the sequential oracle."""
    rng = np.random.default_rng(31 + T)
    n = 9_000_000
    xyz = rng.random((n, 3))
    xyz[: n // 4] = xyz[: n // 4] ** 3  # a dense corner
    xyz[n // 2: n // 2 + 50_000] = xyz[n // 2]  # one repeated point
    bad = rng.integers(0, n, 64)
    xyz[bad[:32]] = [np.nan, 0.5, 2.0]
    xyz[bad[32:]] = [-np.inf, 1.5, 0.25]
    p = _pts(xyz, rng.integers(0, 2**32, n, dtype=np.uint32))
    cfg = LodConfig(leaf_capacity=T, grid_bits=r, max_depth=dmax, chunk_capacity=C)
    dev = to_device(p)
    o = IncrementalOracle(cfg)
    with make_octree(cfg, arena_bytes=6 << 30, max_batch=4_500_000, spill_capacity=10 << 20,
                     backlog_capacity=16 << 20, max_nodes=1 << 20) as tree:
        for k in range(2):
            log(f"case: grouped pass {k}, random cloud, T={T} r={r} Dmax={dmax} C={C}")
            b = slice(k * 4_500_000, (k + 1) * 4_500_000)
            tree.insert(dev[b.start * 16:b.stop * 16])
            o.insert(p[b])
            assert_trees_equal(canonical(tree), o.canonical(), f"after grouped pass {k}")
        st = tree.stats()
    o.close()
    assert st["status_bits"] == 0 and st["num_points"] == n


@pytest.mark.parametrize("order", ["morton", "random"])
def test_aerial_orders_match_sequential_oracle(order):
    """The aerial height field in plain Morton order (few leaves per tile)
    and in random order (nearly every point of a tile in another leaf and
    another claim cell): 3M points in six 500k-point passes, T = 20k, against
    the sequential oracle after every pass."""
    import pointgen

    n, B = 3_000_000, 500_000
    p = pointgen.aerial(n, seed=11, order=order, batch=B)
    cfg = LodConfig(root_size=1024.0, leaf_capacity=20_000)
    dev = to_device(p)
    o = IncrementalOracle(cfg)
    with make_octree(cfg, arena_bytes=2 << 30, max_batch=B, backlog_capacity=4 << 20) as tree:
        for k in range(n // B):
            log(f"case: aerial {order} order, pass {k}")
            b = slice(k * B, (k + 1) * B)
            tree.insert(dev[b.start * 16:b.stop * 16])
            o.insert(p[b])
            assert_trees_equal(canonical(tree), o.canonical(), f"{order}: after pass {k}")
        st = tree.stats()
    o.close()
    assert st["status_bits"] == 0 and st["num_points"] == n and st["num_inner"] > 8


@pytest.mark.parametrize("parts", [[1_000_000], [250_000] * 4, [1, 99_999, 400_000, 500_000],
                                   [333_333, 333_333, 333_334]])
def test_batch_partition_invariance_on_planes(parts):
    import pointgen

    p = pointgen.tiny_planes(1_000_000, seed=3)
    cfg = LodConfig(leaf_capacity=20_000)
    ref = O1.build(p, cfg)
    log(f"case: partition {parts}")
    with make_octree(cfg, arena_bytes=2 << 30) as tree:
        insert_batches(tree, to_device(p), parts)
        assert_trees_equal(canonical(tree), ref, f"parts {parts}")


def test_host_input_and_auto_split_match_device_input():
    import pointgen

    p = pointgen.tiny_planes(200_000, seed=5)
    cfg = LodConfig(leaf_capacity=3_000, grid_bits=6, max_depth=12, chunk_capacity=500)
    ref = O1.build(p, cfg)
    log("case: host pointer input, max_batch 30000")
    with make_octree(cfg, max_batch=30_000) as tree:
        tree.insert(p[:123_457])  # numpy host memory, cut into passes of 30k
        tree.insert(p[123_457:])
        assert tree.stats()["batches"] == 5 + 3
        assert_trees_equal(canonical(tree), ref, "host input")


def test_identical_points_reach_max_depth_on_gpu():
    cfg = LodConfig(leaf_capacity=10, grid_bits=7, max_depth=16, chunk_capacity=8)
    n = 5_000
    p = _pts(np.tile([[0.3, 0.6, 0.9]], (n, 1)), np.arange(n, dtype=np.uint32))
    log("case: identical points")
    with make_octree(cfg) as tree:
        tree.insert(to_device(p[:7]))
        tree.insert(to_device(p[7:]))
        got = canonical(tree)
        st = tree.stats()
    assert_trees_equal(got, O1.build(p, cfg))
    assert len(got.nodes) == 1 + 8 * 16 and got.num_voxels == 16
    assert st["max_rounds"] == 1 + 16 // 4  # one flat round, then 4 levels per round


def test_empty_and_single_point_batches():
    cfg = LodConfig(leaf_capacity=2, grid_bits=2, max_depth=4, chunk_capacity=2)
    rng = np.random.default_rng(12)
    p = _tiny(rng, 40)
    log("case: empty and single batches")
    with make_octree(cfg) as tree:
        tree.insert(to_device(p[:0]))
        for i in range(len(p)):
            tree.insert(to_device(p[i:i + 1]))
            tree.insert(p[:0])
        got = canonical(tree)
    assert_trees_equal(got, O1.build(p, cfg))
    check_invariants(got, p, cfg)


def test_non_power_of_two_domain():
    rng = np.random.default_rng(13)
    cfg = LodConfig(root_min=(-12.7, 3.3, 100.1), root_size=37.9, leaf_capacity=50,
                    grid_bits=4, max_depth=9, chunk_capacity=64)
    xyz = np.array(cfg.root_min) + rng.random((60_000, 3)) ** 2 * 37.9
    p = _pts(xyz, rng.integers(0, 2**32, len(xyz), dtype=np.uint32))
    log("case: non-power-of-two domain")
    with make_octree(cfg) as tree:
        insert_batches(tree, to_device(p), [10_000, 20_000, 30_000])
        assert_trees_equal(canonical(tree), O1.build(p, cfg))


def test_reset_restarts_the_sequence():
    rng = np.random.default_rng(14)
    cfg = LodConfig(leaf_capacity=30, grid_bits=3, max_depth=8)
    p = _tiny(rng, 2_000)
    q = _tiny(rng, 1_500)
    log("case: reset")
    with make_octree(cfg) as tree:
        tree.insert(to_device(p))
        tree.reset()
        tree.insert(to_device(q))
        assert_trees_equal(canonical(tree), O1.build(q, cfg))
        assert tree.stats()["points_inserted"] == 1_500


def test_subtree_snapshots_equal_slices_of_the_whole():
    """simlod_snapshot_subtree returns exactly the whole export's slice for
    that node (nodes-only mode too); missing and malformed paths fail."""
    import pointgen
    from oracle import subtree
    from paper_2310_03567_amd import simlod

    p = pointgen.tiny_planes(300_000, seed=8)
    cfg = LodConfig(leaf_capacity=5_000, grid_bits=5, max_depth=9, chunk_capacity=300)
    log("case: subtree snapshots")
    with make_octree(cfg, arena_bytes=1 << 30) as tree:
        insert_batches(tree, to_device(p), [100_000, 200_000])
        whole = canonical(tree)
        paths = whole.nodes["path"]
        rng = np.random.default_rng(9)
        for path in [1] + rng.choice(paths, 12, replace=False).tolist():
            s = tree.snapshot(int(path))
            want = subtree(whole, int(path))
            assert_trees_equal(canonical_of(s), want, f"path {path}")
            n = tree.snapshot(int(path), nodes_only=True)
            assert n.nodes.tobytes() == s.nodes.tobytes() and len(n.records) == 0
        leaf = int(paths[np.nonzero(whole.nodes["is_leaf"] == 1)[0][0]])
        with pytest.raises(simlod.SimlodError) as e:
            tree.snapshot(leaf * 8 + 1)
        assert e.value.code == simlod.ERR_NOT_FOUND
        for bad in (0, 2, 5, 8 ** 10):  # not a path, or deeper than max_depth
            with pytest.raises(simlod.SimlodError) as e:
                tree.snapshot(bad)
            assert e.value.code == simlod.ERR_INVALID_ARGUMENT


def canonical_of(s):
    from oracle.canonical import CanonicalTree

    return CanonicalTree(nodes=s.nodes, records=s.records, keys=s.keys)


@pytest.mark.parametrize("C", [1, 3, 64, 1000])
def test_chunk_list_reader_equals_table_export(C):
    """Reading every node through its linked chunk list (the renderer's
    access pattern) gives exactly the canonical export, after splits that
    returned chunks to the pool and reused them."""
    import pointgen

    p = pointgen.tiny_planes(120_000, seed=17)
    cfg = LodConfig(leaf_capacity=1_500, grid_bits=5, max_depth=9, chunk_capacity=C)
    log(f"case: chunk lists C={C}")
    with make_octree(cfg, arena_bytes=1 << 30) as tree:
        insert_batches(tree, to_device(p), [5_000, 40_000, 75_000])
        a = tree.snapshot()
        b = tree.snapshot(linked=True)
    assert a.nodes.tobytes() == b.nodes.tobytes()
    assert a.records.tobytes() == b.records.tobytes()
    assert np.array_equal(a.keys, b.keys)
    assert_trees_equal(canonical_of(b), O1.build(p, cfg))


def test_alternating_streams_keep_call_order():
    """Calls on one handle made on different streams run in call order: the
    library makes each new stream wait for the handle's earlier work (the
    passes share the octree's counters, claim table and spill buffers)."""
    import torch

    import pointgen

    p = pointgen.tiny_planes(400_000, seed=31)
    cfg = LodConfig(leaf_capacity=2_000, grid_bits=5, max_depth=10, chunk_capacity=250)
    log("case: alternating torch streams, 16 batches, then a reset on a third stream")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    dev = to_device(p)
    torch.cuda.synchronize()
    with make_octree(cfg, arena_bytes=1 << 30) as tree:
        for k in range(16):
            a, b = k * 25_000, (k + 1) * 25_000
            tree.insert(dev[a * 16:b * 16], streams[k % 2])
        assert_trees_equal(canonical(tree), O1.build(p, cfg), "alternating streams")
        third = torch.cuda.Stream()
        tree.reset(third)
        tree.insert(dev[:150_000 * 16], streams[0])
        tree.insert(dev[150_000 * 16:300_000 * 16], third)
        assert_trees_equal(canonical(tree), O1.build(p[:300_000], cfg), "after reset")


def test_single_node_export_equals_its_slice_of_the_whole():
    import pointgen
    from oracle import subtree
    from paper_2310_03567_amd import simlod

    p = pointgen.tiny_planes(200_000, seed=33)
    cfg = LodConfig(leaf_capacity=3_000, grid_bits=5, max_depth=9, chunk_capacity=300)
    log("case: single-node exports")
    with make_octree(cfg, arena_bytes=1 << 30) as tree:
        insert_batches(tree, to_device(p), [60_000, 140_000])
        whole = canonical(tree)
        for i in list(range(min(40, len(whole.nodes)))):
            path = int(whole.nodes["path"][i])
            s = tree.snapshot_node(path)
            assert len(s.nodes) == 1
            want = subtree(whole, path)
            n0 = want.nodes[0]
            assert (s.nodes[0]["path"], s.nodes[0]["count"], s.nodes[0]["depth"],
                    s.nodes[0]["is_leaf"], s.nodes[0]["first"]) == (
                n0["path"], n0["count"], n0["depth"], n0["is_leaf"], 0)
            r, k = want.node_records(0)
            assert s.records.tobytes() == r.tobytes() and np.array_equal(s.keys, k)
        leaf = int(whole.nodes["path"][np.nonzero(whole.nodes["is_leaf"] == 1)[0][0]])
        with pytest.raises(simlod.SimlodError) as e:
            tree.snapshot_node(leaf * 8 + 3)
        assert e.value.code == simlod.ERR_NOT_FOUND
