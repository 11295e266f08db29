"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

Holds no arithmetic of the matvec method: only the counter-based generator
(SplitMix64 + Box-Muller, see ``synth.c``) and the workload recipes.  Any
entry is a pure function of (seed, stream, index), so a large operator can be
regenerated piecewise.
"""
import ctypes
import os
import subprocess

import numpy as np

from .workloads import SEED, STREAM_BLOCKS, STREAM_M, STREAM_D, STREAM_MTRUE, STREAM_NOISE, WORKLOADS  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.c")
_lib = None


def build(force=False):
    """Compile synth.c into libsynth.so next to it (portable -O2, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        u64, i64 = ctypes.c_uint64, ctypes.c_int64
        vp = ctypes.c_void_p
        lib.synth_normal.argtypes = [u64, u64, u64, i64, vp]
        lib.synth_normal_f32.argtypes = [u64, u64, u64, i64, vp]
        lib.synth_uniform.argtypes = [u64, u64, u64, i64, vp]
        lib.synth_blocks.argtypes = [u64, u64, i64, i64, i64, ctypes.c_double, i64, i64, vp]
        for f in (lib.synth_normal, lib.synth_normal_f32, lib.synth_uniform, lib.synth_blocks):
            f.restype = None
        _lib = lib
    return _lib


def normal(count, stream, offset=0, seed=SEED, dtype=np.float64):
    """``count`` standard normals: entries ``offset .. offset+count-1`` of a stream."""
    lib = _load()
    if dtype == np.float32:
        out = np.empty(int(count), np.float32)
        lib.synth_normal_f32(seed, stream, offset, int(count), out.ctypes.data)
    else:
        out = np.empty(int(count), np.float64)
        lib.synth_normal(seed, stream, offset, int(count), out.ctypes.data)
    return out


def uniform(count, stream, offset=0, seed=SEED):
    """``count`` uniforms in (0, 1)."""
    out = np.empty(int(count), np.float64)
    _load().synth_uniform(seed, stream, offset, int(count), out.ctypes.data)
    return out


def blocks(Nt, Nd, Nm, tau, seed=SEED, stream=STREAM_BLOCKS, k0=0, nk=None, out=None):
    """First block column F_k[s, p] = N(0,1) * exp(-k/tau), shape [nk][Nd][Nm] (FP64).

    Rows k0 .. k0+nk-1 of the full [Nt][Nd][Nm] array; ``tau <= 0`` disables the decay.
    """
    nk = Nt - k0 if nk is None else nk
    if out is None:
        out = np.empty((nk, Nd, Nm), np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.size == nk * Nd * Nm
    _load().synth_blocks(seed, stream, Nt, Nd, Nm, float(tau), k0, nk, out.ctypes.data)
    return out


def vectors(k, Nt, n, stream, seed=SEED, dtype=np.float64):
    """k right-hand sides stacked outermost, time-outer: shape [k][Nt][n]."""
    return normal(k * Nt * n, stream, seed=seed, dtype=dtype).reshape(k, Nt, n)
