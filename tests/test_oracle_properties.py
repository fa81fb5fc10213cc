"""Property tests of the oracle over random tiny batch sequences (hypothesis)."""

from __future__ import annotations

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import POINT_DTYPE, LodConfig, assert_trees_equal
from oracle import definition as O1
from oracle.incremental import build_incremental
from tests.invariants import check_invariants

coord = st.one_of(
    st.sampled_from([0.0, 0.125, 0.25, 0.5, 0.75, 0.999, 1.0, -0.01]),
    st.floats(min_value=0.0, max_value=1.0, width=32),
)


@st.composite
def cases(draw):
    T = draw(st.integers(1, 6))
    r = draw(st.integers(0, 3))
    dmax = draw(st.integers(0, 6))
    n = draw(st.integers(0, 48))
    xyz = draw(st.lists(st.tuples(coord, coord, coord), min_size=n, max_size=n))
    rgba = draw(st.lists(st.integers(0, 2**32 - 1), min_size=n, max_size=n))
    cuts = sorted(draw(st.lists(st.integers(0, n), max_size=5)))
    parts = np.diff([0] + cuts + [n]).tolist()
    return LodConfig(leaf_capacity=T, grid_bits=r, max_depth=dmax, chunk_capacity=3), xyz, rgba, parts


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cases())
def test_batched_sequential_equals_definition(case):
    cfg, xyz, rgba, parts = case
    p = np.zeros(len(xyz), dtype=POINT_DTYPE)
    if len(xyz):
        a = np.asarray(xyz, dtype=np.float32)
        p["x"], p["y"], p["z"] = a[:, 0], a[:, 1], a[:, 2]
        p["rgba"] = np.asarray(rgba, dtype=np.uint32)
    ref = O1.build(p, cfg)
    assert_trees_equal(build_incremental(p, cfg, parts), ref)
    check_invariants(ref, p, cfg, exact=len(p) <= 16)
