"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/simlod.h, and validates arguments on the host before any
device work."""

from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "simlod.h")


def _declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*|simlod_octree\*)\s+(simlod_\w+)\s*\(",
                                 src, re.M)))


@pytest.fixture(scope="module")
def simlod():
    from paper_2310_03567_amd import simlod as m

    return m


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("simlod_create", "simlod_insert_batch", "simlod_snapshot", "simlod_destroy"):
        assert required in names
    assert len(names) >= 10


def test_library_exports_every_declared_function(simlod):
    lib = ctypes.CDLL(simlod.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), f"{name} declared in simlod.h but not exported"
    assert set(_declared_functions()) == set(simlod.EXPORTS)


def test_struct_layouts_match_header(simlod, tmp_path):
    """The ctypes mirrors agree with the C compiler's sizeof/offsetof."""
    structs = {
        "simlod_config": simlod.Config,
        "simlod_snapshot_buffers": simlod.SnapshotBuffers,
        "simlod_stats_data": simlod.StatsData,
        "simlod_kernel_times": simlod.KernelTimes,
        "simlod_server_config": simlod.ServerConfig,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "simlod.h"', "int main(void){"]
    for cname, ct in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append('printf("simlod_node_record %zu\\n", sizeof(simlod_node_record));')
    lines.append('printf("simlod_point %zu\\n", sizeof(simlod_point));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    for cname, ct in structs.items():
        assert int(got[cname]) == ctypes.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(ct, f).offset, f"{cname}.{f}"
    assert int(got["simlod_node_record"]) == simlod.NODE_DTYPE.itemsize == 24
    assert int(got["simlod_point"]) == simlod.POINT_DTYPE.itemsize == 16


def test_default_config_is_the_papers(simlod):
    c = simlod.default_config()
    assert (c.leaf_capacity, c.grid_bits, c.chunk_capacity) == (50_000, 7, 1000)
    assert c.max_depth == 16 and c.root_size == 1.0 and c.backlog_capacity == 10_000_000


@pytest.mark.parametrize("field,value", [
    ("grid_bits", 9), ("max_depth", 22), ("leaf_capacity", 0), ("chunk_capacity", 0),
    ("max_nodes", 8), ("root_size", 0.0), ("root_size", float("inf")), ("root_size", -1.0),
    ("max_batch", 0), ("backlog_capacity", 0),
])
def test_create_rejects_bad_configs_without_touching_the_gpu(simlod, field, value):
    c = simlod.default_config()
    setattr(c, field, value)
    if field == "max_depth":
        c.grid_bits = 2
    h = ctypes.c_void_p(12345)
    rc = simlod.lib.simlod_create(ctypes.byref(c), ctypes.byref(h))
    assert rc == simlod.ERR_INVALID_ARGUMENT
    assert h.value == 12345  # untouched on error


def test_depth_plus_grid_bits_limit(simlod):
    c = simlod.default_config()
    c.max_depth, c.grid_bits = 18, 7  # 25 bits per axis
    h = ctypes.c_void_p()
    assert simlod.lib.simlod_create(ctypes.byref(c), ctypes.byref(h)) == simlod.ERR_INVALID_ARGUMENT


def test_null_arguments(simlod):
    assert simlod.lib.simlod_create(None, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_insert_batch(None, None, 0, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_snapshot(None, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_snapshot_subtree(None, 1, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_stats(None, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_sync(None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_destroy(None) == simlod.OK
    assert simlod.lib.simlod_default_config(None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_group_create(None, 0, 0, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_group_insert(None, None, None, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_group_sync(None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_group_shape(None, None, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_group_destroy(None) == simlod.OK
    assert simlod.lib.simlod_server_create(None, None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_server_destroy(None) == simlod.OK
    assert simlod.lib.simlod_server_drain(None) == simlod.ERR_INVALID_ARGUMENT
    assert simlod.lib.simlod_tune_chunk_capacity(None, None, 0, None, 0, None, None,
                                                 None) == simlod.ERR_INVALID_ARGUMENT


def test_status_strings(simlod):
    for code in range(0, -9, -1):
        s = simlod.status_string(code)
        assert s and s != "unknown status"
    assert simlod.status_string(-99) == "unknown status"
