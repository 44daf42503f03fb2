"""CPU-side checks of the C ABI: the library loads without a GPU and exports
every function include/mos.h declares; the binding mirrors the structs."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mos.h")
LIB = os.path.join(ROOT, "paper_2411_12690_amd", "libmos.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mos_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmos.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_stage_calls():
    fns = declared_functions()
    for name in ("mos_build_cell", "mos_reduce", "mos_solve_array", "mos_reconstruct"):
        assert name in fns


def test_library_exports_every_declared_function(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_covers_every_declared_function():
    from paper_2411_12690_amd import mos
    assert sorted(mos.EXPORTED) == declared_functions()


def test_struct_sizes_match_the_header_layout():
    from paper_2411_12690_amd import mos
    # mos_material: 3 doubles; mos_cell_desc: 3 doubles, 3 int32 (+pad), 2 doubles,
    # 3 materials, 3 int32 and the structure int32, the pad thickness, the skew
    assert ctypes.sizeof(mos.Material) == 24
    assert ctypes.sizeof(mos.CellDesc) == 3 * 8 + 16 + 2 * 8 + 3 * 24 + 16 + 8 + 8
    assert ctypes.sizeof(mos.ArrayDesc) == 4 + 4 + 8 + 8 + 4 + 4 + 8 + 8 + 8 + 4 + 4 + 8 + 4 + 4


def test_context_creation_without_device_reports_an_error(lib):
    # No GPU in this environment: the call must fail cleanly with MOS_EHIP.
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    lib.mos_ctx_create.restype = ctypes.c_int
    lib.mos_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p(1)
    st = lib.mos_ctx_create(0, None, None, ctypes.byref(h))
    assert st == -5 and h.value is None
    assert b"device" in lib.mos_last_error()
