"""Host-side helpers of the benchmark (no GPU)."""

from __future__ import annotations

import bench


def test_busy_seconds_is_the_union_of_the_intervals():
    assert bench.busy_seconds([]) == 0.0
    assert bench.busy_seconds([(1.0, 2.0)]) == 1.0
    # overlapping, nested, touching and disjoint intervals, in any order
    spans = [(5.0, 6.0), (0.0, 2.0), (1.0, 3.0), (1.5, 1.7), (3.0, 4.0), (10.0, 10.5)]
    assert abs(bench.busy_seconds(spans) - (4.0 + 1.0 + 0.5)) < 1e-12


def test_algorithmic_pass_bytes_counts_each_term():
    g = bench.GRID_BYTES
    assert g == 128 ** 3 // 8 == 262_144
    assert bench.algorithmic_pass_bytes(1, 0, 0, 0) == 36
    assert bench.algorithmic_pass_bytes(0, 1, 0, 0) == 40
    assert bench.algorithmic_pass_bytes(0, 0, 1, 0) == 16
    assert bench.algorithmic_pass_bytes(0, 0, 0, 1) == g
    assert bench.algorithmic_pass_bytes(10, 2, 3, 1) == 360 + 80 + 48 + g


def test_kernels_hash_covers_every_device_source():
    import os

    names = sorted(os.path.basename(f) for f in bench.KERNEL_SOURCES)
    assert names == ["kernels.hip", "launch.hpp", "octree_device.hpp"]
    assert all(os.path.exists(f) for f in bench.KERNEL_SOURCES)
    h = bench.kernels_sha256()
    assert len(h) == 64 and h == bench.kernels_sha256()
