"""The C-ABI library loads and exports every function declared in
include/*.h; host-side argument checks work without a GPU (no compute call is
made here)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2607_20766_amd import engine

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*"
                             r"(shape_[a-z0-9_]+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("shape_create", "shape_destroy", "shape_last_error", "shape_estimate",
                     "shape_screen", "shape_alpha_from_radius", "shape_check_data"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = engine.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert lib.shape_version().decode().startswith("shape_is")


def test_struct_layouts_match_header():
    # shape_mols: 2 int32 + int64 + 4 pointers
    assert ctypes.sizeof(engine.ShapeMols) == 8 + 8 + 4 * 8
    assert ctypes.sizeof(engine.ShapeResult) == 18 * 8 + 2 * 8
    assert ctypes.sizeof(engine.ShapeScreenParams) == 4 * 4 + 8 + 8 + 8
    assert ctypes.sizeof(engine.ShapeScreenOut) == 6 * 8
    # shape_gemm_desc: 5 pointers + 6 int64 + 3 int32 + uint32
    assert ctypes.sizeof(engine.ShapeGemmDesc) == 5 * 8 + 6 * 8 + 4 * 4


def test_null_arguments_are_rejected_without_device():
    lib = engine.load_library()
    assert lib.shape_create(None, 0) == -1
    # NULL context: every call returns SHAPE_E_INVAL, no crash
    assert lib.shape_estimate(None, None, None, 10, 10, 0, None, None) == -1
    assert lib.shape_screen(None, None, None, None, 0, None, None, None) == -1
    assert lib.shape_check_data(None, None) == -1
    assert lib.shape_screen_tune(None, None, None, None, 0, None, None, None, None) == -1
    assert lib.shape_screen_set_variant(None, 0) == -1
    assert lib.shape_screen_get_variant(None) == -1
    assert lib.shape_graph_begin(None, None) == -1
    assert lib.shape_graph_end(None, None, None) == -1
    assert lib.shape_graph_launch(None, None, None) == -1
    lib.shape_graph_destroy(None)
    lib.shape_destroy(None)


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="checks the no-device path")
def test_create_without_device_reports_hip_error():
    lib = engine.load_library()
    ctx = ctypes.c_void_p()
    rc = lib.shape_create(ctypes.byref(ctx), 0)
    assert rc == -4
    assert not ctx
    assert b"device" in lib.shape_last_error(None)


def test_profile_ranges_without_a_profiler():
    """The roctx ranges cost nothing and record nothing without a profiler;
    a NULL name is refused."""
    from paper_2607_20766_amd.engine import load_library, profile_range
    lib = load_library()
    with profile_range("outer"):
        with profile_range("inner"):
            pass
    assert lib.shape_range_push(None) == -1
