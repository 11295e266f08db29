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


def test_setup_and_persistence_arguments_rejected(lib):
    h = ctypes.c_void_p()
    assert lib.btoep_create_empty(0, 1, 1, 1, None, ctypes.byref(h)) == 1
    assert lib.btoep_create_empty(4, 1, 1, 9, None, ctypes.byref(h)) == 1
    assert lib.btoep_create_empty(4, 1, 1, 1, None, None) == 1
    assert lib.btoep_set_blocks(None, 0, 1, 0, 1, ctypes.c_void_p(1), 1, 1, 0, 0, None) == 1
    assert lib.btoep_save(None, b"/tmp/x", None) == 1
    assert lib.btoep_load(None, None, ctypes.byref(h)) == 1
    assert lib.btoep_load(b"/tmp/x", None, None) == 1
    assert "I/O" in lib.btoep_status_string(7).decode()


def _header(Nt, Nd, Nm, storage=1, L=None, payload=None, magic=b"BTOEPFH\n", version=1):
    import struct
    N = Nt
    while not _smooth(N):
        N += 1
    L = 2 * N if L is None else L
    if payload is None:
        payload = (L // 2 + 1) * Nd * Nm * {0: 16, 1: 8, 2: 4}[storage]
    return struct.pack("<8sIIqqqqQQ", magic, version, storage, Nt, Nd, Nm, L, payload, 0), payload


def _smooth(n):
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


@pytest.mark.parametrize("case", ["missing", "magic", "version", "length", "truncated", "long", "payload",
                                  "storage", "short"])
def test_malformed_operator_files_rejected_before_device_work(lib, tmp_path, case):
    """btoep_load checks the whole header against the file on the host (status IO = 7)."""
    path = tmp_path / "op.bin"
    hdr, payload = _header(10, 2, 3)
    body = b"\0" * payload
    if case == "magic":
        hdr, _ = _header(10, 2, 3, magic=b"BTOEPFX\n")
    elif case == "version":
        hdr, _ = _header(10, 2, 3, version=2)
    elif case == "length":
        hdr, _ = _header(10, 2, 3, L=24)  # the library pads Nt = 10 to N = 10, L = 20
    elif case == "truncated":
        body = body[:-1]
    elif case == "long":
        body = body + b"\0"
    elif case == "payload":
        hdr, _ = _header(10, 2, 3, payload=payload + 8)
    elif case == "storage":
        hdr, _ = _header(10, 2, 3, storage=5, payload=payload)
    elif case == "short":
        hdr, body = hdr[:40], b""
    if case != "missing":
        path.write_bytes(hdr + body)
    h = ctypes.c_void_p()
    assert lib.btoep_load(os.fsencode(str(path)), None, ctypes.byref(h)) == 7
    assert not h.value


def test_alt_form_arguments_rejected(lib):
    assert lib.btoep_alt_prepare(None, 1, None) == 1
    assert lib.btoep_alt_apply(None, 0, 1, None, None, None) == 1


def test_stepwise_cg_arguments_rejected(lib):
    """The caller-memory CG entry points check their arguments on the host."""
    dev, host = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.btoep_cg_state_size(None, None, 1, ctypes.byref(dev), ctypes.byref(host)) == 1
    assert lib.btoep_cg_workspace_size(None, None, 1, ctypes.byref(dev)) == 1
    h = ctypes.c_void_p()
    assert lib.btoep_cg_begin(None, None, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), 1e-6, 1e-3,
                              ctypes.c_void_p(256), 1 << 20, ctypes.c_void_p(8), 1 << 10, None,
                              ctypes.byref(h)) == 1
    assert lib.btoep_cg_begin(None, None, 1, None, None, 1e-6, 1e-3, None, 0, None, 0, None, None) == 1
    for f in (lib.btoep_cg_refine, lib.btoep_cg_update, lib.btoep_cg_poll):
        assert f(None, None) == 1
    x, hx = ctypes.c_void_p(), ctypes.c_void_p()
    assert lib.btoep_cg_residual_vectors(None, ctypes.byref(x), ctypes.byref(hx)) == 1
    ready = ctypes.c_int()
    assert lib.btoep_cg_report(None, ctypes.byref(ready), None) == 1
    assert lib.btoep_cg_end(None) == 1


def test_gemm_tuning_arguments_rejected(lib):
    assert lib.btoep_set_gemm(None, 0) == 1
    assert lib.btoep_set_gemm_variants(None, 8, 0, 0) == 1
    assert lib.btoep_autotune_gemm(None, 8, 1, 3, None, None) == 1


def test_bandwidth_calibration_arguments_rejected(lib):
    """Sizes below 1 MiB, no repetitions or missing outputs are rejected before any device call."""
    out = [ctypes.c_double() for _ in range(3)]
    refs = [ctypes.byref(o) for o in out]
    for fn in (lib.btoep_read_bandwidth, lib.btoep_write_bandwidth):
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_double)] * 3
        assert fn(1024, 3, None, *refs) == 1
        assert fn(1 << 24, 0, None, *refs) == 1
        assert fn(1 << 24, 3, None, None, refs[1], refs[2]) == 1
