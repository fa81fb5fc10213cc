"""Brute-force checker of the octree invariants, independent of both oracles.

Given the cumulative point sequence and a canonical tree, it re-derives every
fact from the points alone, node by node, without recursion over the tree's
own partition:

* the node set is a full octree: the root has path 1, every inner node has all
  eight children, depths match path lengths, preorder with octant order;
* every key appears in exactly one leaf, whose region contains the point,
  with its record bit-identical to the input; leaf lists are sorted by key;
* no leaf above the maximum depth holds more than T points, and every inner
  node's region holds more than T points (section "Expanding the Octree");
* an inner node has exactly one voxel per occupied cell of its R^3 grid, none
  for empty cells (section "Voxel Sampling Grid"), coloured by the point with
  the smallest key in the cell, placed at the cell centre;
* chunk bookkeeping: ceil(count / C) chunks per node (section "Allocating
  Chunks") -- returned as a total for comparison with a library's counters.

Integer coordinates are computed here with exact rational arithmetic
(``fractions``) for small inputs, so the checker does not share the
floating-point formulation of the oracles; for larger inputs a float32
numpy path is used after it has been cross-checked against the exact one.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np

from oracle.canonical import POINT_DTYPE, CanonicalTree, LodConfig


def _f32(v) -> np.float32:
    return np.float32(v)


def quantize_exact(v: float, vmin: float, cfg: LodConfig) -> int:
    """Integer coordinate via IEEE float32 semantics emulated with Fractions.

    fl32(a - b) and fl32(a * b) are computed as the exact rational result
    rounded to the nearest float32 (ties to even), the definition of IEEE
    binary32 arithmetic.
    """
    if np.isnan(v):
        return 0
    a = _round_f32(Fraction(float(np.float32(v))) - Fraction(float(np.float32(vmin)))) \
        if np.isfinite(v) else None
    if a is None:
        return 0 if v < 0 else (1 << cfg.K) - 1
    scale = _round_f32(Fraction(2**cfg.K) / Fraction(float(np.float32(cfg.root_size))))
    u = _round_f32(a * scale)
    if u is None:  # overflow to +-inf
        return (1 << cfg.K) - 1 if a > 0 else 0
    if u < 0:
        return 0
    q = u.numerator // u.denominator
    return min(q, (1 << cfg.K) - 1)


def _round_f32(x: Fraction):
    """Round a rational to the nearest binary32 value (ties to even).

    Returns None on overflow.
    """
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    ax = -x if x < 0 else x
    # exponent e with 2^e <= ax < 2^(e+1)
    e = ax.numerator.bit_length() - ax.denominator.bit_length()
    if Fraction(2) ** e > ax:
        e -= 1
    elif Fraction(2) ** (e + 1) <= ax:
        e += 1
    e = max(e, -126)  # subnormal range
    ulp = Fraction(2) ** (e - 23)
    m = ax / ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * ulp
    if r >= Fraction(2) ** 128:
        return None
    return sign * r


def quantize_np(v: np.ndarray, vmin, cfg: LodConfig) -> np.ndarray:
    v = np.asarray(v, dtype=np.float32)
    scale = np.float32(np.float32(2.0**cfg.K) / np.float32(cfg.root_size))
    with np.errstate(invalid="ignore", over="ignore"):
        u = (v - np.float32(vmin)) * scale
        fl = np.floor(np.where(u >= 0, u, 0)).astype(np.float64)
    fl = np.minimum(fl, (1 << cfg.K) - 1)
    fl[~(u >= 0)] = 0
    return fl.astype(np.int64)


def centre_exact(g: int, vmin: float, cfg: LodConfig, depth: int) -> np.float32:
    h = Fraction(float(np.float32(cfg.root_size))) / (2 ** (cfg.grid_bits + depth))
    prod = _round_f32((g + Fraction(1, 2)) * h)
    s = _round_f32(Fraction(float(np.float32(vmin))) + prod)
    return np.float32(float(s))


def path_octants(path: int):
    octs = []
    p = int(path)
    while p > 1:
        octs.append(p & 7)
        p >>= 3
    return octs[::-1]


def check_invariants(tree: CanonicalTree, points: np.ndarray, cfg: LodConfig,
                     exact: bool | None = None) -> dict:
    """Raises AssertionError on the first violated invariant; returns stats."""
    pts = np.ascontiguousarray(points, dtype=POINT_DTYPE)
    n = len(pts)
    if exact is None:
        exact = n <= 400
    if exact:
        q = np.array([[quantize_exact(float(p[a]), cfg.root_min[i], cfg)
                       for i, a in enumerate("xyz")] for p in pts], dtype=np.int64).reshape(n, 3)
    else:
        q = np.stack([quantize_np(pts[a], cfg.root_min[i], cfg) for i, a in enumerate("xyz")], 1)
    nodes = tree.nodes
    K, Dmax, R, T = cfg.K, cfg.max_depth, cfg.R, cfg.leaf_capacity

    # --- structure: preorder walk must reproduce the node list exactly
    paths = [int(p) for p in nodes["path"]]
    assert paths and paths[0] == 1, "root path must be 1"
    pos = {p: i for i, p in enumerate(paths)}
    assert len(pos) == len(paths), "duplicate paths"
    order = []
    stack = [1]
    while stack:
        p = stack.pop()
        order.append(p)
        i = pos.get(p)
        assert i is not None, f"missing node path {p}"
        if nodes["is_leaf"][i] == 0:
            stack.extend(p * 8 + o for o in range(7, -1, -1))
    assert order == paths, "node list is not the preorder of a full octree"
    written = 0
    for i, nd in enumerate(nodes):
        assert int(nd["depth"]) == len(path_octants(nd["path"])), f"depth of node {i}"
        assert int(nd["first"]) == written, f"records of node {i} not contiguous"
        written += int(nd["count"])
    assert written == len(tree.records) == len(tree.keys)

    seen = np.zeros(n, dtype=np.int32)
    chunks = 0
    levels = 0
    for i, nd in enumerate(nodes):
        depth = int(nd["depth"])
        levels = max(levels, depth + 1)
        octs = path_octants(nd["path"])
        sel = np.ones(n, dtype=bool)
        for d, o in enumerate(octs):
            b = K - 1 - d
            for a in range(3):
                sel &= ((q[:, a] >> b) & 1) == ((o >> a) & 1)
        members = np.nonzero(sel)[0]  # keys are positions
        recs, keys = tree.node_records(i)
        cnt = int(nd["count"])
        chunks += -(-cnt // cfg.chunk_capacity)
        assert np.all(np.diff(keys.astype(np.int64)) > 0), f"node {i}: keys not sorted"
        if nd["is_leaf"]:
            assert depth == Dmax or cnt <= T, f"leaf {i} at depth {depth} holds {cnt} > T"
            assert np.array_equal(keys.astype(np.int64), members), f"leaf {i}: wrong point set"
            assert recs.tobytes() == pts[members].tobytes(), f"leaf {i}: records differ"
            seen[members] += 1
        else:
            assert depth < Dmax, f"inner node {i} at max depth"
            assert len(members) > T, f"inner node {i} region holds only {len(members)} <= T"
            shift = Dmax - depth
            g = q[members] >> shift
            cell = (g & (R - 1))
            lin = cell[:, 0] + R * (cell[:, 1] + R * cell[:, 2])
            firsts = {}
            for j, c in enumerate(lin):
                if int(c) not in firsts:
                    firsts[int(c)] = j  # members are in key order
            exp_keys = np.array(sorted(members[j] for j in firsts.values()), dtype=np.int64)
            assert np.array_equal(keys.astype(np.int64), exp_keys), \
                f"inner {i}: representatives differ ({len(keys)} vs {len(exp_keys)} voxels)"
            for r_i, k in enumerate(keys):
                k = int(k)
                assert recs["rgba"][r_i] == pts["rgba"][k], f"inner {i}: voxel colour"
                gk = q[k] >> shift
                for a, ax in enumerate("xyz"):
                    if exact:
                        c = centre_exact(int(gk[a]), cfg.root_min[a], cfg, depth)
                    else:
                        h = np.float32(np.ldexp(np.float32(cfg.root_size), -(cfg.grid_bits + depth)))
                        c = np.float32(cfg.root_min[a]) + (np.float32(gk[a]) + np.float32(0.5)) * h
                    assert recs[ax][r_i].tobytes() == np.float32(c).tobytes(), \
                        f"inner {i}: voxel {r_i} {ax} centre {recs[ax][r_i]} != {c}"
    assert np.all(seen == 1), "some point is not in exactly one leaf"
    return {"chunks": chunks, "levels": levels, "nodes": len(nodes)}
