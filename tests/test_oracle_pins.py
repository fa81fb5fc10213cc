"""Pins of the CPU oracle to facts other than itself (no GPU needed).

* integer coordinates and voxel centres against an exact rational emulation
  of IEEE binary32 arithmetic (tests/invariants.py) and closed forms;
* the hand-worked example in tests/golden (section "Incrementally Updating
  the Octree", update figure, T = 5, chunks of 2);
* closed forms: n <= T, n > T identical points, a 1-cell grid, a lattice;
* O1 (recursive definition) against O2 (sequential C inserter) exhaustively
  over tiny inputs, each also run through the brute-force invariant checker;
* batch-partition and permutation invariance; the per-update voxel bound
  (section "Voxel Sampling");
* planted mistakes in the oracle are caught by these pins.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

from oracle import POINT_DTYPE, LodConfig, assert_trees_equal, subtree, trees_equal
from oracle import definition as O1
from oracle.incremental import IncrementalOracle, build_incremental
from tests.golden_util import check_against_expected, load_fig_update
from tests.invariants import centre_exact, check_invariants, quantize_exact


def _points(xyz, rgba=None):
    xyz = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    p = np.zeros(len(xyz), dtype=POINT_DTYPE)
    p["x"], p["y"], p["z"] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    p["rgba"] = np.arange(len(xyz), dtype=np.uint32) * 0x01010101 + 7 if rgba is None else rgba
    return p


# ---------------------------------------------------------------- coordinates

def test_quantize_power_of_two_closed_form():
    rng = np.random.default_rng(0)
    for size_exp in (-3, 0, 1, 10):
        size = 2.0**size_exp
        cfg = LodConfig(root_size=size)
        x = (rng.random(2000) * size).astype(np.float32)
        q = O1.quantize(x, 0.0, cfg)
        exp = [int(Fraction(float(v)) * 2**cfg.K / Fraction(size)) for v in x]
        assert q.tolist() == exp


def test_quantize_boundaries_and_specials():
    cfg = LodConfig()  # K = 23, unit cube
    K = cfg.K
    ks = np.array([0, 1, 2, 12345, (1 << K) - 2, (1 << K) - 1], dtype=np.int64)
    x = (ks.astype(np.float64) / 2**K).astype(np.float32)
    assert O1.quantize(x, 0.0, cfg).tolist() == ks.tolist()  # boundary -> upper cell
    sp = np.array([np.nan, -np.inf, np.inf, -0.5, -0.0, 1.0, 2.0, np.float32(1) - np.float32(2**-24)],
                  dtype=np.float32)
    assert O1.quantize(sp, 0.0, cfg).tolist() == [0, 0, (1 << K) - 1, 0, 0, (1 << K) - 1,
                                                  (1 << K) - 1, (1 << K) - 1]
    for v, e in zip(sp.tolist(), O1.quantize(sp, 0.0, cfg).tolist()):
        assert quantize_exact(v, 0.0, cfg) == e


@pytest.mark.parametrize("mn,size", [(-1.3, 3.7), (100.25, 1000.0), (0.1, 0.3), (-5.0, 16.0)])
def test_quantize_matches_ieee_emulation(mn, size):
    cfg = LodConfig(root_min=(mn, mn, mn), root_size=size)
    rng = np.random.default_rng(1)
    x = (np.float32(mn) + rng.random(300) * np.float32(size) * 1.02 - 0.01 * size).astype(np.float32)
    q = O1.quantize(x, mn, cfg)
    assert q.tolist() == [quantize_exact(float(v), mn, cfg) for v in x]
    order = np.argsort(x)
    assert np.all(np.diff(q[order].astype(np.int64)) >= 0)  # monotone


@pytest.mark.parametrize("mn,size", [(0.0, 1.0), (-1.3, 3.7), (100.25, 1000.0), (0.0, 1024.0)])
def test_voxel_centre_matches_ieee_emulation(mn, size):
    cfg = LodConfig(root_min=(mn, mn, mn), root_size=size)
    rng = np.random.default_rng(2)
    for depth in (0, 1, 5, 15):
        g = rng.integers(0, 1 << (cfg.grid_bits + depth), 50).astype(np.uint32)
        c = O1.voxel_centre(g, mn, cfg, depth)
        assert [v.tobytes() for v in c] == [centre_exact(int(v), mn, cfg, depth).tobytes() for v in g]
        if mn == 0.0 and size in (1.0, 1024.0):  # exact closed form
            h = Fraction(size) / 2 ** (cfg.grid_bits + depth)
            assert [Fraction(float(v)) for v in c] == [(int(v) + Fraction(1, 2)) * h for v in g]


# ------------------------------------------------------------ golden example

@pytest.mark.parametrize("impl", ["O1", "O2"])
def test_fig_update_hand_example(impl):
    cfg, batches, expected = load_fig_update()
    if impl == "O2":
        o = IncrementalOracle(cfg)
    inserted = []
    for b, e in zip(batches, expected):
        inserted.append(b)
        allp = np.concatenate(inserted)
        if impl == "O1":
            tree = O1.build(allp, cfg)
        else:
            o.insert(b)
            tree = o.canonical()
        check_against_expected(tree, allp, e)
        st = check_invariants(tree, allp, cfg)
        assert st["chunks"] == e["chunks"]
        assert tree.nodes["count"].sum() == sum(len(n["keys"]) for n in e["nodes"])


# -------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [0, 1, 17, 50])
def test_at_most_T_points_is_one_leaf(n):
    cfg = LodConfig(leaf_capacity=50)
    rng = np.random.default_rng(n)
    p = _points(rng.random((n, 3)))
    for tree in (O1.build(p, cfg), build_incremental(p, cfg)):
        assert len(tree.nodes) == 1 and tree.nodes[0]["is_leaf"] == 1
        assert tree.nodes[0]["count"] == n and tree.num_voxels == 0
        assert tree.records.tobytes() == p.tobytes()


@pytest.mark.parametrize("dmax,r", [(0, 7), (1, 2), (4, 3), (16, 7)])
def test_identical_points_reach_max_depth(dmax, r):
    T = 3
    n = 9
    cfg = LodConfig(leaf_capacity=T, grid_bits=r, max_depth=dmax)
    xyz = np.tile(np.array([[0.3, 0.6, 0.9]], dtype=np.float32), (n, 1))
    rgba = np.arange(n, dtype=np.uint32) + 100
    p = _points(xyz, rgba)
    q = [int(v) for v in (O1.quantize(xyz[0], 0.0, cfg))]
    for tree in (O1.build(p, cfg), build_incremental(p, cfg)):
        assert len(tree.nodes) == 1 + 8 * dmax
        assert tree.num_voxels == dmax
        inner = tree.nodes["is_leaf"] == 0
        assert np.all(tree.nodes["count"][inner] == 1)
        vox_idx = tree.nodes["first"][inner]
        assert np.all(tree.keys[vox_idx] == 0) and np.all(tree.records["rgba"][vox_idx] == 100)
        full = tree.nodes[(tree.nodes["is_leaf"] == 1) & (tree.nodes["count"] > 0)]
        assert len(full) == 1 and full[0]["depth"] == dmax and full[0]["count"] == n
        path = 1
        for d in range(dmax):
            b = cfg.K - 1 - d
            path = path * 8 + sum(((q[a] >> b) & 1) << a for a in range(3))
        assert full[0]["path"] == path


def test_single_cell_grid_gives_node_centres():
    cfg = LodConfig(leaf_capacity=4, grid_bits=0, max_depth=5)
    rng = np.random.default_rng(3)
    p = _points(rng.random((300, 3)) ** 2)
    tree = O1.build(p, cfg)
    assert_trees_equal(tree, build_incremental(p, cfg))
    check_invariants(tree, p, cfg)
    for i, nd in enumerate(tree.nodes):
        if nd["is_leaf"]:
            continue
        recs, keys = tree.node_records(i)
        assert len(keys) == 1
        octs = []
        path = int(nd["path"])
        while path > 1:
            octs.append(path & 7)
            path >>= 3
        octs.reverse()
        lo = [Fraction(0)] * 3
        size = Fraction(1)
        for o in octs:
            size /= 2
            lo = [lo[a] + size * ((o >> a) & 1) for a in range(3)]
        centre = [lo[a] + size / 2 for a in range(3)]
        assert [Fraction(float(recs[a][0])) for a in "xyz"] == centre
        region_keys = _keys_in_region(p, cfg, octs)
        assert keys[0] == min(region_keys)


def _keys_in_region(p, cfg, octs):
    sel = np.ones(len(p), bool)
    for d, o in enumerate(octs):
        for a, ax in enumerate("xyz"):
            q = O1.quantize(p[ax], 0.0, cfg)
            sel &= ((q >> (cfg.K - 1 - d)) & 1) == ((o >> a) & 1)
    return np.nonzero(sel)[0]


def test_lattice_closed_form():
    """(2R)^3 lattice at depth-1 cell centres, R = 4, Dmax = 2, T = 7.

    Root: 512 points, one voxel per root cell (64), each cell holding 8
    points.  Depth 1: 8 inner nodes with 64 points, one per cell, so each
    voxel is exactly its point.  Depth 2 = Dmax: 64 leaves of 8 points.
    """
    cfg = LodConfig(leaf_capacity=7, grid_bits=2, max_depth=2)
    idx = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1).reshape(-1, 3)
    xyz = (idx + 0.5) / 8.0
    rng = np.random.default_rng(4)
    perm = rng.permutation(len(xyz))
    p = _points(xyz[perm], rng.integers(0, 2**32, len(xyz), dtype=np.uint32))
    for tree in (O1.build(p, cfg), build_incremental(p, cfg, [100, 200, 212])):
        assert len(tree.nodes) == 73
        inner = tree.nodes["is_leaf"] == 0
        assert inner.sum() == 9 and tree.num_voxels == 64 + 8 * 64
        assert tree.nodes[0]["count"] == 64
        leaves = tree.nodes[~inner]
        assert np.all(leaves["count"] == 8) and np.all(leaves["depth"] == 2)
        for i in np.nonzero(inner)[0][1:]:
            recs, keys = tree.node_records(i)
            for j, k in enumerate(keys):
                assert recs[j].tobytes() == p[k].tobytes()  # centre == the point itself
        # root voxels: min key among the 8 lattice points of each root cell
        recs, keys = tree.node_records(0)
        cell_of = (idx[perm] // 2)
        lin = cell_of[:, 0] + 4 * (cell_of[:, 1] + 4 * cell_of[:, 2])
        exp = sorted(int(np.nonzero(lin == c)[0].min()) for c in range(64))
        assert keys.tolist() == exp


# --------------------------------------------------- O1 vs O2, exhaustively

def _tiny_case(rng, n):
    mode = rng.integers(0, 3)
    if mode == 0:
        xyz = rng.random((n, 3))
    elif mode == 1:  # lattice-clustered, many duplicates and boundary hits
        xyz = rng.integers(0, 8, (n, 3)) / 8.0
    else:  # clustered near a corner to force depth
        xyz = rng.random((n, 3)) ** 4
    if n and rng.random() < 0.2:  # a few out-of-domain and NaN coordinates
        xyz[rng.integers(0, n)] = [np.nan, -3.0, 7.0]
    return _points(xyz, rng.integers(0, 2**32, n, dtype=np.uint32))


def test_definition_equals_sequential_inserter_exhaustive_tiny():
    rng = np.random.default_rng(5)
    cases = 0
    for T in (1, 2, 5):
        for r in (0, 1, 2):
            for dmax in range(5):
                for _ in range(6):
                    n = int(rng.integers(0, 65))
                    cfg = LodConfig(leaf_capacity=T, grid_bits=r, max_depth=dmax, chunk_capacity=2)
                    p = _tiny_case(rng, n)
                    a = O1.build(p, cfg)
                    b = build_incremental(p, cfg)
                    assert_trees_equal(a, b, f"T={T} r={r} Dmax={dmax} n={n}")
                    check_invariants(a, p, cfg, exact=n <= 24)
                    cases += 1
    assert cases == 270


def test_partition_invariance():
    rng = np.random.default_rng(6)
    cfg = LodConfig(leaf_capacity=5, grid_bits=2, max_depth=6)
    p = _points(rng.random((400, 3)) ** 3, rng.integers(0, 2**32, 400, dtype=np.uint32))
    ref = O1.build(p, cfg)
    for parts in ([400], [1] * 400, [7, 0, 93, 300], [200, 200], [399, 1]):
        assert_trees_equal(build_incremental(p, cfg, parts), ref, f"parts {parts[:4]}")


def test_region_subtrees_equal_subtrees_of_the_definition():
    """O2 fed only one node's region (keys of the whole sequence kept) gives
    that node's subtree of O1's whole-sequence octree, for every node: the
    route by which subtrees of clouds too large for one oracle run are
    checked."""
    rng = np.random.default_rng(15)
    checked = 0
    for T, r, dmax, n in ((3, 2, 5, 500), (1, 1, 4, 120), (8, 3, 7, 2_000), (5, 0, 3, 300)):
        cfg = LodConfig(leaf_capacity=T, grid_bits=r, max_depth=dmax, chunk_capacity=3)
        p = _points(rng.random((n, 3)) ** 3, rng.integers(0, 2**32, n, dtype=np.uint32))
        full = O1.build(p, cfg)
        paths = full.nodes["path"]
        pick = paths if len(paths) <= 40 else rng.choice(paths, 40, replace=False)
        for path in pick:
            o = IncrementalOracle(cfg)
            for part in np.array_split(p, 3):
                o.insert_region(part, int(path))
            got = o.region_subtree(int(path))
            assert o.total == n
            o.close()
            want = subtree(full, int(path))
            assert_trees_equal(got, want, f"T={T} r={r} Dmax={dmax} path={int(path)}")
            checked += 1
    assert checked > 60
    o = IncrementalOracle(LodConfig(max_depth=2))
    for bad in (0, 2, 7, 8 * 8 * 8 * 8 + 1):  # no leading 1 / too deep
        with pytest.raises(ValueError):
            o.insert_region(p[:10], bad)
    o.close()


def test_subtree_slicing_matches_a_fresh_preorder():
    """``subtree`` of the root is the tree itself; the subtrees of the root's
    children tile its nodes and records in order."""
    rng = np.random.default_rng(16)
    cfg = LodConfig(leaf_capacity=4, grid_bits=2, max_depth=6)
    p = _points(rng.random((700, 3)) ** 2, rng.integers(0, 2**32, 700, dtype=np.uint32))
    t = O1.build(p, cfg)
    assert_trees_equal(subtree(t, 1), t)
    nodes, recs = 1, int(t.nodes["count"][0])
    for o in range(8):
        s = subtree(t, 8 + o)
        assert s.nodes["path"][0] == 8 + o and s.nodes["first"][0] == 0
        nodes += len(s.nodes)
        recs += len(s.records)
        assert all(int(q) >> (3 * (int(d) - 1)) == 8 + o
                   for q, d in zip(s.nodes["path"], s.nodes["depth"]))
    assert nodes == len(t.nodes) and recs == len(t.records)
    leaf = int(t.nodes["path"][np.nonzero(t.nodes["is_leaf"] == 1)[0][0]])
    assert subtree(t, leaf * 8 + 3) is None  # below a leaf: no such node


def test_permutation_invariance_with_uniform_colour():
    rng = np.random.default_rng(7)
    cfg = LodConfig(leaf_capacity=6, grid_bits=1, max_depth=5)
    xyz = rng.random((300, 3)) ** 2
    p = _points(xyz, np.full(300, 0xAABBCCDD, np.uint32))
    a = O1.build(p, cfg)
    b = O1.build(p[rng.permutation(300)], cfg)
    for f in ("path", "depth", "is_leaf", "count", "first"):
        assert np.array_equal(a.nodes[f], b.nodes[f])
    for i in range(len(a.nodes)):
        ra, _ = a.node_records(i)
        rb, _ = b.node_records(i)
        assert sorted(r.tobytes() for r in ra) == sorted(r.tobytes() for r in rb)


def test_voxels_per_update_bounded_by_levels_times_work():
    """Each point of the work list (batch plus spilled points) visits at most
    levels-1 inner nodes and creates at most one voxel in each (section
    "Voxel Sampling" bounds the backlog by (levels - 1) x batch size; spilled
    points are re-sampled too, so they join the batch in the bound)."""
    rng = np.random.default_rng(8)
    cfg = LodConfig(leaf_capacity=20, grid_bits=3, max_depth=8)
    o = IncrementalOracle(cfg)
    prev = o.canonical()
    allp = []
    for b in range(12):
        n = int(rng.integers(1, 150))
        pts = _points(rng.random((n, 3)) ** 3, rng.integers(0, 2**32, n, dtype=np.uint32))
        allp.append(pts)
        o.insert(pts)
        cur = o.canonical()
        before = {int(nd["path"]): nd for nd in prev.nodes}
        spilled = sum(int(before[int(nd["path"])]["count"]) for nd in cur.nodes
                      if nd["is_leaf"] == 0 and int(nd["path"]) in before
                      and before[int(nd["path"])]["is_leaf"] == 1)
        levels = int(cur.nodes["depth"].max()) + 1
        v = o.voxels_created_last
        assert v == cur.num_voxels - prev.num_voxels
        assert v <= (levels - 1) * (n + spilled)
        prev = cur
    assert_trees_equal(prev, O1.build(np.concatenate(allp), cfg))


# ----------------------------------------------- planted mistakes are caught

def _golden_and_invariants_pass():
    cfg, batches, expected = load_fig_update()
    allp = np.concatenate(batches)
    tree = O1.build(allp, cfg)
    try:
        check_against_expected(tree, allp, expected[1])
        check_invariants(tree, allp, cfg)
    except AssertionError:
        return False
    rng = np.random.default_rng(9)
    for cfg2 in (LodConfig(leaf_capacity=3, grid_bits=1, max_depth=4),
                 LodConfig(leaf_capacity=2, grid_bits=0, max_depth=3)):
        p = _points(rng.random((40, 3)) ** 2, rng.integers(0, 2**32, 40, dtype=np.uint32))
        try:
            check_invariants(O1.build(p, cfg2), p, cfg2, exact=True)
        except AssertionError:
            return False
    return True


def test_pins_catch_planted_mistakes(monkeypatch):
    assert _golden_and_invariants_pass()
    real_quant = O1.quantize
    real_centre = O1.voxel_centre
    mutants = {
        "ceil instead of floor": lambda v, mn, cfg: np.minimum(
            real_quant(v, mn, cfg) + ((np.asarray(v, np.float32) - np.float32(mn)) * cfg.scale
                                      % 1 != 0), (1 << cfg.K) - 1).astype(np.uint32),
        "off-by-one cell": lambda v, mn, cfg: np.minimum(real_quant(v, mn, cfg) + 1,
                                                         (1 << cfg.K) - 1).astype(np.uint32),
    }
    for name, fn in mutants.items():
        monkeypatch.setattr(O1, "quantize", fn)
        assert not _golden_and_invariants_pass(), name
        monkeypatch.setattr(O1, "quantize", real_quant)
    monkeypatch.setattr(O1, "voxel_centre", lambda g, mn, cfg, d: real_centre(g, mn, cfg, d + 1))
    assert not _golden_and_invariants_pass(), "wrong centre depth"
    monkeypatch.setattr(O1, "voxel_centre", real_centre)

    # split at >= T instead of > T, and first-come by largest key
    cfg, batches, expected = load_fig_update()
    allp = np.concatenate(batches)
    import dataclasses
    # ">= T" splits a leaf holding exactly T points; the n == T closed form
    # (test_at_most_T_points_is_one_leaf) pins the strict rule.
    p_t = _points(np.random.default_rng(10).random((50, 3)))
    bad = O1.build(p_t, dataclasses.replace(LodConfig(leaf_capacity=50), leaf_capacity=49))
    assert len(bad.nodes) > 1
    rev = O1.build(allp, cfg, keys=np.arange(len(allp))[::-1].copy())
    assert not trees_equal(rev, O1.build(allp, cfg))
    with pytest.raises(AssertionError):
        check_against_expected(rev, allp, expected[1])
