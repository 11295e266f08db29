"""The C-ABI library loads here (no GPU) and exports every entry point the header declares."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "btoep.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(btoep_[a-z_A-Z]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2407_13066_amd as bt
    from paper_2407_13066_amd import build
    if build.stale():
        build.build()
    return bt.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["btoep_create", "btoep_destroy", "btoep_query", "btoep_workspace_size", "btoep_apply_F",
              "btoep_apply_FT", "btoep_apply_H", "btoep_apply_batched", "btoep_cg_solve",
              "btoep_status_string", "btoep_last_error"]:
        assert n in names, n


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_status_strings(lib):
    import paper_2407_13066_amd as bt
    assert bt.btoep_status_string(0) == "ok"
    assert "workspace" in bt.btoep_status_string(6)
    assert bt.btoep_status_string(99) == "unknown status"


def test_invalid_arguments_rejected_before_any_launch(lib):
    """Argument checks run on the host and need no device."""
    h = ctypes.c_void_p()
    assert lib.btoep_create(0, 1, 1, ctypes.c_void_p(1), 0, 1, None, ctypes.byref(h)) == 1
    assert lib.btoep_create(4, 1, 1, None, 0, 1, None, ctypes.byref(h)) == 1
    assert lib.btoep_create(4, 1, 1, ctypes.c_void_p(1), 0, 7, None, ctypes.byref(h)) == 1
    assert lib.btoep_create(4, 1, 1, ctypes.c_void_p(1), 0, 1, None, None) == 1
    assert lib.btoep_apply_F(None, 1, None, None, None, 0, None) == 1
    assert lib.btoep_destroy(None) == 1
    assert lib.btoep_query(None, None) == 1
    assert lib.btoep_graph_launch(None, None, None, None) == 1
    assert lib.btoep_graph_destroy(None) == 1
    assert lib.btoep_set_fft(None, 0) == 1
    g = ctypes.c_void_p()
    assert lib.btoep_graph_create(None, 2, 1, 1.0, 1.0, ctypes.c_void_p(8), 1 << 20, ctypes.byref(g)) == 1
    assert lib.btoep_graph_create(None, 2, 1, 1.0, 1.0, None, 0, None) == 1
