"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every entry point the header declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import pytest

import paper_2302_13524_amd as tm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "tm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = tm.load()
    names = header_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tm.EXPORTED)


def test_grid_support_table():
    lib = tm.load()
    for n1, n2 in [(128, 64), (64, 128), (32, 32), (8, 8), (64, 64), (64, 32), (1, 1024)]:
        assert lib.tm_grid_supported(n1, n2) == 1
    for n1, n2 in [(3, 8), (128, 128), (256, 64), (0, 8), (-4, 4)]:
        assert lib.tm_grid_supported(n1, n2) == 0


def test_launch_configuration_table():
    # digit orders everywhere; eight values per thread and twice the rows per
    # workgroup on the workload grids, within 1024 (512 for twice the rows) threads
    for n1, n2 in [(8, 8), (64, 128), (1, 1024)]:
        assert [c for c in range(8) if tm.tm_config_info(n1, n2, c)] == [0, 1]
    assert tm.tm_config_info(32, 32, 0) == (256, 4, 16)
    assert tm.tm_config_info(32, 32, 2) == (256, 2, 8)
    assert tm.tm_config_info(32, 32, 6) == (512, 4, 8)
    assert tm.tm_config_info(64, 64, 4) == (512, 2, 16)
    assert tm.tm_config_info(64, 64, 6) is None
    assert tm.tm_config_info(128, 64, 2) == (1024, 1, 8)
    assert tm.tm_config_info(128, 64, 4) is None
    for n1, n2 in [(32, 32), (64, 32), (64, 64), (128, 64)]:
        for c in range(8):
            sh = tm.tm_config_info(n1, n2, c)
            if sh is None:
                continue
            wg, rpw, ept = sh
            assert wg * ept == rpw * n1 * n2  # whole rows per workgroup
            assert ept in (8, 16) and wg <= 1024 and wg % 64 == 0
    for bad in [(-1, 32, 32), (8, 32, 32), (0, 3, 8), (0, 128, 128)]:
        assert tm.tm_config_info(bad[1], bad[2], bad[0]) is None


def test_null_context_is_rejected():
    lib = tm.load()
    d = tm.tm_dims(8, 8, 4, 1)
    assert lib.tm_forward(None, d, None, None, 0, 0, None, None) == tm.TM_EINVAL
    assert lib.tm_retrieve(None, d, None, None, None, None, None, None) == tm.TM_EINVAL
    assert lib.tm_destroy(None) == tm.TM_EINVAL


def test_create_reports_missing_device_or_bad_index():
    lib = tm.load()
    h = ctypes.c_void_p()
    rc = lib.tm_create(ctypes.byref(h), 99)
    assert rc in (tm.TM_EINVAL, tm.TM_EHIP)
    assert lib.tm_last_error(None)
    assert not h.value
    assert lib.tm_create(None, 0) == tm.TM_EINVAL


def test_struct_layouts_match_header():
    assert ctypes.sizeof(tm.tm_dims) == 16
    assert ctypes.sizeof(tm.tm_retrieve_opts) == 40
    assert ctypes.sizeof(tm.tm_defocus_dims) == 20
    assert ctypes.sizeof(tm.tm_optics) == 32
    assert tm.ROW_STATS_BYTES == 24
