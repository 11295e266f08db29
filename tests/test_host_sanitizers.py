"""Host paths of the C-ABI library under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host code (argument validation, the operator-file header parser, workspace and
state layouts) is rebuilt with -fsanitize=address,undefined on the host side only (device code is
unchanged) and driven, in a separate process with the sanitizer runtime preloaded, through every
argument check and malformed-operator-file case of test_abi.py; any sanitizer report fails."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "asan")

DRIVER = r'''
import ctypes, os, struct, sys, tempfile
sys.path.insert(0, os.environ["BTOEP_ROOT"])
import paper_2407_13066_amd as bt
lib = bt.load_library(os.environ["BTOEP_ASAN_LIB"])
from tests import test_abi as t
t.test_invalid_arguments_rejected_before_any_launch(lib)
t.test_setup_and_persistence_arguments_rejected(lib)
t.test_alt_form_arguments_rejected(lib)
t.test_stepwise_cg_arguments_rejected(lib)
t.test_gemm_tuning_arguments_rejected(lib)
t.test_status_strings(lib)
import pathlib
for case in ["missing", "magic", "version", "length", "truncated", "long", "payload", "storage", "short"]:
    with tempfile.TemporaryDirectory() as d:
        t.test_malformed_operator_files_rejected_before_device_work(lib, pathlib.Path(d), case)
# headers naming absurd sizes (overflowing products) are refused before any allocation
for Nt, Nd, Nm in [(2**40, 2, 3), (10, 2**40, 3), (10, 2, 2**62), (-5, 2, 3), (10, 0, 3)]:
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "op.bin")
        hdr = struct.pack("<8sIIqqqqQQ", b"BTOEPFH\n", 1, 1, Nt, Nd, Nm, 2 * max(Nt, 1), 2**63, 0)
        open(p, "wb").write(hdr + b"\0" * 64)
        h = ctypes.c_void_p()
        assert lib.btoep_load(os.fsencode(p), None, ctypes.byref(h)) == 7, (Nt, Nd, Nm)
print("sanitized host paths ok")
'''


def _runtime():
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return c[-1] if c else None


def _build():
    from paper_2407_13066_amd import build as b
    os.makedirs(OUT, exist_ok=True)
    objs = []
    base = os.path.join(ROOT, "_build", "btoep")
    if not all(os.path.exists(os.path.join(base, s.replace(".hip", ".o"))) for s in b.SOURCES):
        b.build()
    flags = [f for f in b.HIPCC_FLAGS if f not in ("-shared", "-O3")] + ["-O1", "-g"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", b.CSRC]
    for src in b.SOURCES:
        if src == "api.hip":
            obj = os.path.join(OUT, "api.o")
            subprocess.check_call([b.hipcc()] + flags + san + inc + ["-c", os.path.join(b.CSRC, src), "-o", obj])
            objs.append(obj)
        else:
            objs.append(os.path.join(base, src.replace(".hip", ".o")))
    so = os.path.join(OUT, "libbtoep_asan.so")
    subprocess.check_call([b.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan"] + san +
                          ["-o", so] + objs)
    return so


@pytest.mark.timeout(600)
def test_host_paths_clean_under_asan_and_ubsan():
    rt = _runtime()
    if rt is None:
        pytest.skip("no sanitizer runtime in this ROCm installation")
    so = _build()
    env = dict(os.environ, LD_PRELOAD=rt, BTOEP_ASAN_LIB=so, BTOEP_ROOT=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "sanitized host paths ok" in out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
