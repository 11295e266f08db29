"""MI355X-native FFT matvecs with block lower-triangular Toeplitz operators.

A thin ctypes binding over ``libbtoep.so`` (HIP, gfx950), the C interface declared in
``include/btoep.h``.  Functions carry the C names; they only marshal arguments
(torch device tensors, the current HIP stream) -- every step of the computation runs in
the library's kernels.  There is no fallback: when the library is missing or cannot be
loaded every call raises.

Layouts (time-outer, right-hand sides outermost):
  blocks [Nt][Nd][Nm] FP64,  m [k][Nt][Nm],  d [k][Nt][Nd]
Vector dtype: float64 for an operator stored as "f64", float32 for "f32" and "bf16".
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbtoep.so")

BTOEP_OK = 0
BTOEP_ERR_NOT_CONVERGED = 5
BTOEP_ERR_WORKSPACE_TOO_SMALL = 6
BTOEP_ERR_IO = 7
ORDER = {"column": 0, "last_row": 1}
STORAGE = {"f64": 0, "f32": 1, "bf16": 2}
WHICH = {"F": 0, "FT": 1, "H": 2, "CG": 3}
MAX_BATCH = 64
STATIC_SCRATCH_BYTES = 128 << 20   # BTOEP_STATIC_SCRATCH_BYTES

_lib = None


class BtoepError(RuntimeError):
    def __init__(self, status, what, detail=""):
        self.status = status
        msg = "%s failed: %s" % (what, btoep_status_string(status))
        if detail:
            msg += " [%s]" % detail
        super().__init__(msg)


class _Info(ctypes.Structure):
    _fields_ = [("Nt", ctypes.c_int64), ("Nd", ctypes.c_int64), ("Nm", ctypes.c_int64),
                ("L", ctypes.c_int64), ("nfreq", ctypes.c_int64), ("ldF", ctypes.c_int64),
                ("storage", ctypes.c_int), ("vector", ctypes.c_int), ("fhat_bytes", ctypes.c_size_t),
                ("device", ctypes.c_int)]


class CgOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_outer", ctypes.c_int), ("max_inner", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("check_every", ctypes.c_int), ("use_graph", ctypes.c_int)]


class CgResult(ctypes.Structure):
    _fields_ = [("inner_iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("nvar", ctypes.c_int), ("var_n", ctypes.c_int), ("var_c", ctypes.c_int),
                ("ms_n", ctypes.c_double * 8), ("ms_c", ctypes.c_double * 8), ("fft_four_step", ctypes.c_int),
                ("ms_fft", ctypes.c_double * 2)]


class GemmTuneResult(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("nvar_n", ctypes.c_int), ("nvar_c", ctypes.c_int), ("var_n", ctypes.c_int),
                ("var_c", ctypes.c_int), ("split", ctypes.c_int), ("ms_n", (ctypes.c_double * 8) * 2),
                ("ms_c", (ctypes.c_double * 8) * 2)]


def load_library(path=LIB_PATH):
    """Load libbtoep.so (raises OSError when it is missing or unloadable)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError("libbtoep.so not built at %s (run __graft_entry__.build())" % path)
    # torch first: the library then binds to the HIP runtime torch has loaded, so the process
    # holds one runtime (with the library loaded first, calls into it from a process whose
    # torch brings its own runtime have failed with "no ROCm-capable device")
    _torch()
    lib = ctypes.CDLL(path)
    vp, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "btoep_create": ([i64, i64, i64, vp, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)], st),
        "btoep_create_empty": ([i64, i64, i64, ctypes.c_int, vp, ctypes.POINTER(vp)], st),
        "btoep_set_blocks": ([vp, i64, i64, i64, i64, vp, i64, i64, ctypes.c_int, ctypes.c_int, vp], st),
        "btoep_save": ([vp, ctypes.c_char_p, vp], st),
        "btoep_load": ([ctypes.c_char_p, vp, ctypes.POINTER(vp)], st),
        "btoep_alt_prepare": ([vp, ctypes.c_int, vp], st),
        "btoep_alt_apply": ([vp, ctypes.c_int, ctypes.c_int, vp, vp, vp], st),
        "btoep_destroy": ([vp], st),
        "btoep_query": ([vp, ctypes.POINTER(_Info)], st),
        "btoep_workspace_size": ([vp, ctypes.c_int, i64, ctypes.POINTER(sz)], st),
        "btoep_apply_F": ([vp, i64, vp, vp, vp, sz, vp], st),
        "btoep_apply_FT": ([vp, i64, vp, vp, vp, sz, vp], st),
        "btoep_apply_H": ([vp, i64, dbl, dbl, vp, vp, vp, sz, vp], st),
        "btoep_apply_batched": ([vp, ctypes.c_int, i64, ctypes.POINTER(vp), ctypes.POINTER(vp), dbl, dbl, vp, sz,
                                 vp], st),
        "btoep_apply_static": ([vp, ctypes.c_int, i64, dbl, dbl, vp, vp, vp], st),
        "btoep_graph_create": ([vp, ctypes.c_int, i64, dbl, dbl, vp, sz, ctypes.POINTER(vp)], st),
        "btoep_graph_launch": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp], st),
        "btoep_graph_destroy": ([vp], st),
        "btoep_cg_solve": ([vp, vp, i64, dbl, dbl, vp, vp, ctypes.POINTER(CgOpts), ctypes.POINTER(CgResult), vp,
                            sz, vp], st),
        "btoep_autotune": ([vp, ctypes.c_int, vp, ctypes.POINTER(TuneResult)], st),
        "btoep_set_tuning": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int], st),
        "btoep_set_gemm": ([vp, ctypes.c_int], st),
        "btoep_set_gemm_variants": ([vp, i64, ctypes.c_int, ctypes.c_int], st),
        "btoep_autotune_gemm": ([vp, i64, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(GemmTuneResult)], st),
        "btoep_set_fft": ([vp, i64], st),
        "btoep_profile_enable": ([vp, ctypes.c_int], st),
        "btoep_profile_read": ([vp, ctypes.POINTER(KernelTime), ctypes.c_int, ctypes.POINTER(ctypes.c_int)], st),
        "btoep_cg_start": ([vp, i64, dbl, dbl, vp, vp, dbl, vp, ctypes.POINTER(vp)], st),
        "btoep_cg_vectors": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp)], st),
        "btoep_cg_update": ([vp, vp], st),
        "btoep_cg_poll": ([vp, vp], st),
        "btoep_cg_status": ([vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)], st),
        "btoep_cg_end": ([vp], st),
        "btoep_cg_state_size": ([vp, vp, i64, ctypes.POINTER(sz), ctypes.POINTER(sz)], st),
        "btoep_cg_begin": ([vp, vp, i64, vp, vp, dbl, dbl, vp, sz, vp, sz, vp, ctypes.POINTER(vp)], st),
        "btoep_cg_residual_vectors": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp)], st),
        "btoep_cg_refine": ([vp, vp], st),
        "btoep_cg_report": ([vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(CgResult)], st),
        "btoep_cg_workspace_size": ([vp, vp, i64, ctypes.POINTER(sz)], st),
        "btoep_read_bandwidth": ([sz, ctypes.c_int, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                  ctypes.POINTER(dbl)], st),
        "btoep_write_bandwidth": ([sz, ctypes.c_int, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                   ctypes.POINTER(dbl)], st),
        "btoep_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "btoep_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check(status, what, op=None):
    if status != BTOEP_OK:
        lib = load_library()
        detail = lib.btoep_last_error(op).decode() if lib else ""
        raise BtoepError(status, what, detail)


def btoep_status_string(status):
    return load_library().btoep_status_string(int(status)).decode()


def btoep_last_error(op=None):
    return load_library().btoep_last_error(op.handle if isinstance(op, Op) else op).decode()


class Op:
    """Owning handle of a created operator (destroyed with btoep_destroy or on collection)."""

    def __init__(self, handle, info):
        self.handle = handle
        self.info = info
        self.Nt, self.Nd, self.Nm = info["Nt"], info["Nd"], info["Nm"]
        self.storage = info["storage"]

    @property
    def vector_dtype(self):
        torch = _torch()
        return torch.float64 if self.storage == "f64" else torch.float32

    def destroy(self):
        if self.handle:
            load_library().btoep_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def btoep_create(blocks, storage="f32", stream=None):
    """Set up the Fourier-space operator from the first block column ``blocks`` [Nt][Nd][Nm] (FP64).

    ``blocks`` is a numpy array (host) or a torch float64 tensor (host or device).
    """
    import numpy as np
    lib = load_library()
    torch = _torch()
    if isinstance(blocks, np.ndarray):
        arr = np.ascontiguousarray(blocks, dtype=np.float64)
        ptr, where, shape, keep = arr.ctypes.data, 0, arr.shape, arr
    else:
        t = blocks
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("blocks must be a contiguous float64 tensor")
        ptr, where, shape, keep = t.data_ptr(), (1 if t.is_cuda else 0), tuple(t.shape), t
    if len(shape) != 3:
        raise ValueError("blocks must have shape [Nt][Nd][Nm]")
    Nt, Nd, Nm = shape
    h = ctypes.c_void_p()
    st = lib.btoep_create(Nt, Nd, Nm, ctypes.c_void_p(ptr), where, STORAGE[storage], _stream(stream),
                          ctypes.byref(h))
    del keep
    _check(st, "btoep_create")
    return Op(h, btoep_query(h))


def btoep_create_empty(Nt, Nd, Nm, storage="f32", stream=None):
    """An operator of the given shape with all blocks zero; fill it with btoep_set_blocks."""
    h = ctypes.c_void_p()
    _check(load_library().btoep_create_empty(int(Nt), int(Nd), int(Nm), STORAGE[storage], _stream(stream),
                                             ctypes.byref(h)), "btoep_create_empty")
    return Op(h, btoep_query(h))


def btoep_set_blocks(op, s0, p0, blocks, order="column", stream=None):
    """Transform and store sensors s0.. x parameters p0.. from ``blocks`` [Nt][ns][np] (FP64).

    ``order`` "column": blocks[t] = F_t (first block column); "last_row": blocks[t] = F_{Nt-1-t}
    (last block row).  ``blocks`` is a numpy array or a torch float64 tensor (host or device),
    possibly a strided view whose last axis is contiguous.
    """
    import numpy as np
    torch = _torch()
    if isinstance(blocks, np.ndarray):
        if blocks.dtype != np.float64:
            raise ValueError("blocks must be float64")
        if blocks.ndim != 3 or blocks.strides[2] != 8 or blocks.strides[0] % 8 or blocks.strides[1] % 8:
            raise ValueError("blocks must be [Nt][ns][np] with a contiguous last axis")
        ptr, where, shape = blocks.ctypes.data, 0, blocks.shape
        ld_t, ld_s = blocks.strides[0] // 8, blocks.strides[1] // 8
    else:
        t = blocks
        if t.dtype != torch.float64 or t.dim() != 3 or t.stride(2) != 1:
            raise ValueError("blocks must be a float64 [Nt][ns][np] tensor with a contiguous last axis")
        ptr, where, shape = t.data_ptr(), (1 if t.is_cuda else 0), tuple(t.shape)
        ld_t, ld_s = t.stride(0), t.stride(1)
    if shape[0] != op.Nt:
        raise ValueError("blocks has %d time rows, the operator %d" % (shape[0], op.Nt))
    ns, np_ = shape[1], shape[2]
    if ns == 1:
        ld_s = max(ld_s, np_)
    _check(load_library().btoep_set_blocks(op.handle, int(s0), int(ns), int(p0), int(np_), ctypes.c_void_p(ptr),
                                           int(ld_t), int(ld_s), ORDER[order], where, _stream(stream)),
           "btoep_set_blocks", op.handle)


def btoep_save(op, path, stream=None):
    """Write the stored Fourier-space operator to ``path``."""
    _check(load_library().btoep_save(op.handle, os.fsencode(path), _stream(stream)), "btoep_save", op.handle)


def btoep_load(path, stream=None):
    """A new operator holding the Fourier-space operator saved in ``path``."""
    h = ctypes.c_void_p()
    _check(load_library().btoep_load(os.fsencode(path), _stream(stream), ctypes.byref(h)), "btoep_load")
    return Op(h, btoep_query(h))


def btoep_alt_prepare(op, mode=1, stream=None):
    """Build the SOTI copy of the stored operator for the appendix form (mode 0: products then
    a separate reduction, as in the paper's appendix; mode 1: fused)."""
    _check(load_library().btoep_alt_prepare(op.handle, int(mode), _stream(stream)), "btoep_alt_prepare", op.handle)


def btoep_alt_apply(op, which, x, mode=1, out=None, stream=None):
    """F (which "F": x = m [Nt][Nm]) or F^T ("FT": x = d [Nt][Nd]) by the appendix form; one
    right-hand side.  For comparison with btoep_apply_F / btoep_apply_FT."""
    torch = _torch()
    if which not in ("F", "FT"):
        raise ValueError("which must be 'F' or 'FT'")
    tin = (op.Nt, op.Nm) if which == "F" else (op.Nt, op.Nd)
    tout = (op.Nt, op.Nd) if which == "F" else (op.Nt, op.Nm)
    if not x.is_cuda or x.dtype != op.vector_dtype or not x.is_contiguous() or tuple(x.shape) != tin:
        raise ValueError("input must be a contiguous %s CUDA tensor of shape %s" % (op.vector_dtype, list(tin)))
    if out is None:
        out = torch.empty(tout, dtype=x.dtype, device=x.device)
    if not out.is_cuda or out.dtype != x.dtype or not out.is_contiguous() or tuple(out.shape) != tout:
        raise ValueError("out must be a contiguous %s CUDA tensor of shape %s" % (x.dtype, list(tout)))
    _check(load_library().btoep_alt_apply(op.handle, WHICH[which], int(mode), ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), _stream(stream)),
           "btoep_alt_apply", op.handle)
    return out


def btoep_destroy(op):
    op.destroy()


def btoep_query(op):
    lib = load_library()
    info = _Info()
    h = op.handle if isinstance(op, Op) else op
    _check(lib.btoep_query(h, ctypes.byref(info)), "btoep_query")
    names = {v: k for k, v in STORAGE.items()}
    return dict(Nt=info.Nt, Nd=info.Nd, Nm=info.Nm, L=info.L, nfreq=info.nfreq, ldF=info.ldF,
                storage=names[info.storage], vector=names[info.vector], fhat_bytes=info.fhat_bytes,
                device=info.device)


def btoep_workspace_size(op, which, k=1):
    n = ctypes.c_size_t()
    _check(load_library().btoep_workspace_size(op.handle, WHICH[which], int(k), ctypes.byref(n)),
           "btoep_workspace_size", op.handle)
    return n.value


def _vec(op, t, tail, name, dtype=None, single=False):
    """Check a vector argument: a contiguous CUDA tensor on the operator's device, of the
    operator's vector dtype (or ``dtype``), shaped [k]+tail (or tail, read as k = 1; only
    tail when ``single``).  Returns the [k]+tail view."""
    torch = _torch()
    dtype = op.vector_dtype if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
    t3 = t.unsqueeze(0) if t.dim() == 2 else t
    if t3.dim() != 3 or tuple(t3.shape[1:]) != tuple(tail) or (single and t3.shape[0] != 1):
        raise ValueError("%s has shape %s, expected %s%s" % (name, tuple(t.shape), "" if single else "[k]",
                                                             list(tail)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    if t.device.index != op.info["device"]:
        raise ValueError("%s is on cuda:%s, the operator on cuda:%d" % (name, t.device.index, op.info["device"]))
    return t3


def _io_tails(op, which):
    """Trailing shapes of the input and output vectors of an apply."""
    n_in = op.Nd if which == "FT" else op.Nm
    n_out = op.Nd if which == "F" else op.Nm
    return (op.Nt, n_in), (op.Nt, n_out)


def _ws(ws):
    if ws is None:
        return ctypes.c_void_p(None), 0
    return ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()


def btoep_apply_F(op, m, d=None, ws=None, stream=None):
    """d = F m.  m: [k][Nt][Nm] (or [Nt][Nm]); returns d [k][Nt][Nd] (same leading form)."""
    torch = _torch()
    squeeze = m.dim() == 2
    m3 = _vec(op, m, (op.Nt, op.Nm), "m")
    k = m3.shape[0]
    if d is None:
        d = torch.empty((k, op.Nt, op.Nd), dtype=m.dtype, device=m.device)
    d3 = _vec(op, d, (op.Nt, op.Nd), "d")
    wp, wn = _ws(ws)
    _check(load_library().btoep_apply_F(op.handle, k, ctypes.c_void_p(m3.data_ptr()),
                                        ctypes.c_void_p(d3.data_ptr()), wp, wn, _stream(stream)),
           "btoep_apply_F", op.handle)
    return d3[0] if squeeze else d


def btoep_apply_FT(op, d, m=None, ws=None, stream=None):
    """m = F^T d.  d: [k][Nt][Nd]; returns m [k][Nt][Nm]."""
    torch = _torch()
    squeeze = d.dim() == 2
    d3 = _vec(op, d, (op.Nt, op.Nd), "d")
    k = d3.shape[0]
    if m is None:
        m = torch.empty((k, op.Nt, op.Nm), dtype=d.dtype, device=d.device)
    m3 = _vec(op, m, (op.Nt, op.Nm), "m")
    wp, wn = _ws(ws)
    _check(load_library().btoep_apply_FT(op.handle, k, ctypes.c_void_p(d3.data_ptr()),
                                         ctypes.c_void_p(m3.data_ptr()), wp, wn, _stream(stream)),
           "btoep_apply_FT", op.handle)
    return m3[0] if squeeze else m


def btoep_apply_H(op, m, noise_prec=1.0, prior_prec=1.0, out=None, ws=None, stream=None):
    """Hm = F^T (noise_prec F m) + prior_prec m."""
    torch = _torch()
    squeeze = m.dim() == 2
    m3 = _vec(op, m, (op.Nt, op.Nm), "m")
    k = m3.shape[0]
    if out is None:
        out = torch.empty((k, op.Nt, op.Nm), dtype=m.dtype, device=m.device)
    o3 = _vec(op, out, (op.Nt, op.Nm), "out")
    wp, wn = _ws(ws)
    _check(load_library().btoep_apply_H(op.handle, k, float(noise_prec), float(prior_prec),
                                        ctypes.c_void_p(m3.data_ptr()), ctypes.c_void_p(o3.data_ptr()),
                                        wp, wn, _stream(stream)),
           "btoep_apply_H", op.handle)
    return o3[0] if squeeze else out


def btoep_read_bandwidth(nbytes, reps=5, stream=None):
    """Streaming-read rate of one device array of ``nbytes`` (btoep_read_bandwidth)."""
    ms, best, mean = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().btoep_read_bandwidth(int(nbytes), int(reps), _stream(stream), ctypes.byref(ms),
                                               ctypes.byref(best), ctypes.byref(mean)), "btoep_read_bandwidth")
    return {"best_ms": round(ms.value, 4), "best_GBs": round(best.value, 1), "mean_GBs": round(mean.value, 1)}


def btoep_write_bandwidth(nbytes, reps=5, stream=None):
    """Streaming-write rate of one device array of ``nbytes`` (btoep_write_bandwidth)."""
    ms, best, mean = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().btoep_write_bandwidth(int(nbytes), int(reps), _stream(stream), ctypes.byref(ms),
                                                ctypes.byref(best), ctypes.byref(mean)), "btoep_write_bandwidth")
    return {"best_ms": round(ms.value, 4), "best_GBs": round(best.value, 1), "mean_GBs": round(mean.value, 1)}


def btoep_apply_static(op, which, x, out, noise_prec=1.0, prior_prec=1.0, stream=None):
    """F, F^T or H (``which``) of x into ``out`` with the library's static device scratch as the
    workspace (btoep_apply_static: no allocation; calls on one device must not overlap)."""
    tin, tout = _io_tails(op, which)
    x3 = _vec(op, x, tin, "x")
    o3 = _vec(op, out, tout, "out")
    if o3.shape[0] != x3.shape[0]:
        raise ValueError("x and out hold different numbers of right-hand sides")
    _check(load_library().btoep_apply_static(op.handle, WHICH[which], x3.shape[0], float(noise_prec),
                                             float(prior_prec), ctypes.c_void_p(x3.data_ptr()),
                                             ctypes.c_void_p(o3.data_ptr()), _stream(stream)),
           "btoep_apply_static", op.handle)
    return out


def btoep_apply_batched(op, which, ins, outs, noise_prec=1.0, prior_prec=1.0, ws=None, stream=None):
    """Pointer-array apply: ins[r] / outs[r] are separate device tensors ([Nt][Nm] or [Nt][Nd])."""
    k = len(ins)
    if k != len(outs) or k > MAX_BATCH:
        raise ValueError("need len(ins) == len(outs) <= %d" % MAX_BATCH)
    if which not in ("F", "FT", "H"):
        raise ValueError("which must be 'F', 'FT' or 'H'")
    tin, tout = _io_tails(op, which)
    for r in range(k):
        _vec(op, ins[r], tin, "ins[%d]" % r, single=True)
        _vec(op, outs[r], tout, "outs[%d]" % r, single=True)
    PA = ctypes.c_void_p * max(k, 1)
    pin = PA(*[t.data_ptr() for t in ins])
    pout = PA(*[t.data_ptr() for t in outs])
    wp, wn = _ws(ws)
    _check(load_library().btoep_apply_batched(op.handle, WHICH[which], k, pin, pout, float(noise_prec),
                                              float(prior_prec), wp, wn, _stream(stream)),
           "btoep_apply_batched", op.handle)
    return outs


def btoep_cg_solve(op_lo, op_hi, b, x, noise_prec, prior_prec, rtol=1e-8, max_outer=10, max_inner=1000,
                   inner_rtol=1e-4, check_every=4, ws=None, stream=None, raise_on_not_converged=False,
                   use_graph=True):
    """Solve H x = b (FP64 b, x of shape [k][Nt][Nm] on the device; x is the initial guess).

    ``use_graph`` replays each inner iteration from a captured HIP graph.
    Returns (status, [CgResult per right-hand side]).
    """
    torch = _torch()
    tail = (op_lo.Nt, op_lo.Nm)
    if tuple(x.shape) != tuple(b.shape):
        raise ValueError("x has shape %s, b %s: they must match" % (tuple(x.shape), tuple(b.shape)))
    b3 = _vec(op_lo, b, tail, "b", dtype=torch.float64)
    _vec(op_lo, x, tail, "x", dtype=torch.float64)
    k = b3.shape[0]
    opts = CgOpts(rtol, max_outer, max_inner, inner_rtol, check_every, 1 if use_graph else 0)
    res = (CgResult * k)()
    wp, wn = _ws(ws)
    st = load_library().btoep_cg_solve(op_lo.handle, op_hi.handle if op_hi is not None else None, k,
                                       float(noise_prec), float(prior_prec), ctypes.c_void_p(b.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()), ctypes.byref(opts), res, wp, wn,
                                       _stream(stream))
    if st not in (BTOEP_OK, BTOEP_ERR_NOT_CONVERGED) or (st != BTOEP_OK and raise_on_not_converged):
        _check(st, "btoep_cg_solve", op_lo.handle)
    return st, [dict(inner_iters=r.inner_iters, outer_iters=r.outer_iters, matvecs=r.matvecs,
                     converged=bool(r.converged), rel_residual=r.rel_residual) for r in res]


def btoep_profile_enable(op, enable=True):
    """Start (and reset) or stop per-kernel HIP-event timing on this operator."""
    _check(load_library().btoep_profile_enable(op.handle, 1 if enable else 0), "btoep_profile_enable", op.handle)


def btoep_profile_read(op):
    """{kernel name: (launches, total ms)} since profiling was enabled (waits for the events)."""
    buf = (KernelTime * 16)()
    n = ctypes.c_int()
    _check(load_library().btoep_profile_read(op.handle, buf, 16, ctypes.byref(n)), "btoep_profile_read", op.handle)
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(n.value)}


def btoep_autotune(op, reps=5, stream=None):
    """Time the single-vector product variants (and, where both apply, the two transform
    modes) on this operator and keep the fastest.

    Returns {"var_n", "var_c", "ms_n": [...], "ms_c": [...], "fft_four_step", "ms_fft": [single,
    four-step]} (milliseconds per launch).
    """
    r = TuneResult()
    _check(load_library().btoep_autotune(op.handle, int(reps), _stream(stream), ctypes.byref(r)),
           "btoep_autotune", op.handle)
    return {"var_n": r.var_n, "var_c": r.var_c, "ms_n": [round(r.ms_n[i], 4) for i in range(r.nvar)],
            "ms_c": [round(r.ms_c[i], 4) for i in range(r.nvar)], "fft_four_step": bool(r.fft_four_step),
            "ms_fft": [round(r.ms_fft[0], 4), round(r.ms_fft[1], 4)]}


def btoep_set_fft(op, n1=0):
    """Transform mode: 0 automatic, n1 > 1 four-step with first factor n1, n1 < 0 single-pass."""
    _check(load_library().btoep_set_fft(op.handle, int(n1)), "btoep_set_fft", op.handle)


def btoep_set_gemm(op, split):
    """FP32 storage: several-right-hand-side products on the BF16 matrix cores with the
    three-term split (``split`` true) or on the FP32 matrix cores."""
    _check(load_library().btoep_set_gemm(op.handle, 1 if split else 0), "btoep_set_gemm", op.handle)


def btoep_set_gemm_variants(op, k, var_n, var_c):
    """Pin the matrix-core kernel variants used for k right-hand sides (its bucket)."""
    _check(load_library().btoep_set_gemm_variants(op.handle, int(k), int(var_n), int(var_c)),
           "btoep_set_gemm_variants", op.handle)


def btoep_autotune_gemm(op, k, allow_split=True, reps=3, stream=None):
    """Time the matrix-core kernel variants (and, for FP32 storage with ``allow_split``, the
    BF16-matrix-core mode) for k right-hand sides and keep the fastest for k's bucket.

    Returns {"k", "nvar_n", "nvar_c", "var_n", "var_c", "split", "ms_n": {mode: [ms per variant]},
    "ms_c": ...}."""
    r = GemmTuneResult()
    _check(load_library().btoep_autotune_gemm(op.handle, int(k), 1 if allow_split else 0, int(reps),
                                              _stream(stream), ctypes.byref(r)), "btoep_autotune_gemm", op.handle)
    modes = [0, 1] if (allow_split and op.storage == "f32") else [int(r.split)]
    return {"k": r.k, "nvar_n": r.nvar_n, "nvar_c": r.nvar_c, "var_n": r.var_n, "var_c": r.var_c,
            "split": bool(r.split),
            "ms_n": {("split" if m else "fp32" if op.storage == "f32" else "bf16"):
                     [round(r.ms_n[m][v], 4) for v in range(r.nvar_n)] for m in modes},
            "ms_c": {("split" if m else "fp32" if op.storage == "f32" else "bf16"):
                     [round(r.ms_c[m][v], 4) for v in range(r.nvar_c)] for m in modes}}


def btoep_set_tuning(op, var_n, var_c, use_mfma=True):
    """Pin the single-vector kernel variants and the multi-vector kernel choice."""
    _check(load_library().btoep_set_tuning(op.handle, int(var_n), int(var_c), 1 if use_mfma else 0),
           "btoep_set_tuning", op.handle)


class CgState:
    """Stepwise CG (btoep_cg_*): the caller applies H_lo to ``p`` into ``Ap`` before each
    update and, with a refinement operator, H_hi to ``x`` into ``Hx`` before each refine.

    ``keep`` holds the caller-side memory (device and pinned host tensors) of a state made by
    btoep_cg_begin, so that it lives as long as the state."""

    def __init__(self, op, handle, k, op_hi=None, keep=None):
        self.op, self.op_hi, self.handle, self.k, self.keep = op, op_hi, handle, k, keep
        p, ap = ctypes.c_void_p(), ctypes.c_void_p()
        _check(load_library().btoep_cg_vectors(handle, ctypes.byref(p), ctypes.byref(ap)), "btoep_cg_vectors",
               op.handle)
        self.p_ptr, self.ap_ptr = p.value, ap.value
        self.vec_bytes = op.Nt * op.Nm * (8 if op.storage == "f64" else 4)
        self.x_ptr = self.hx_ptr = None
        if op_hi is not None:
            x, hx = ctypes.c_void_p(), ctypes.c_void_p()
            _check(load_library().btoep_cg_residual_vectors(handle, ctypes.byref(x), ctypes.byref(hx)),
                   "btoep_cg_residual_vectors", op.handle)
            self.x_ptr, self.hx_ptr = x.value, hx.value

    def p(self, r):
        return self.p_ptr + r * self.vec_bytes

    def ap(self, r):
        return self.ap_ptr + r * self.vec_bytes

    def x(self, r):
        """FP64 iterate of right-hand side r (refined state only)."""
        return self.x_ptr + r * self.op.Nt * self.op.Nm * 8

    def hx(self, r):
        """FP64 array that receives H_hi x of right-hand side r (refined state only)."""
        return self.hx_ptr + r * self.op.Nt * self.op.Nm * 8

    def tensors(self):
        """Torch views [k][Nt][Nm] of the state's p and Ap arrays (device memory the state owns;
        valid until end()), for callers that add terms of their own to H p -- e.g. a general
        prior operator applied by the caller, with H run at prior_prec = 0."""
        torch = _torch()
        typestr = "<f8" if self.op.storage == "f64" else "<f4"
        shape = (self.k, self.op.Nt, self.op.Nm)

        class _View:
            def __init__(self, ptr):
                self.__cuda_array_interface__ = {"shape": shape, "typestr": typestr, "data": (ptr, False),
                                                 "version": 3, "strides": None}
        return (torch.as_tensor(_View(self.p_ptr), device="cuda"),
                torch.as_tensor(_View(self.ap_ptr), device="cuda"))

    def end(self):
        if self.handle:
            load_library().btoep_cg_end(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.end()
        except Exception:
            pass


def btoep_cg_start(op, b, x, rtol, noise_prec=1.0, prior_prec=1.0, stream=None):
    """Start stepwise CG for the stacked right-hand sides b (x receives the solution, zeroed here)."""
    b3 = _vec(op, b, (op.Nt, op.Nm), "b")
    x3 = _vec(op, x, (op.Nt, op.Nm), "x")
    h = ctypes.c_void_p()
    _check(load_library().btoep_cg_start(op.handle, b3.shape[0], float(noise_prec), float(prior_prec),
                                         ctypes.c_void_p(b3.data_ptr()), ctypes.c_void_p(x3.data_ptr()),
                                         float(rtol), _stream(stream), ctypes.byref(h)), "btoep_cg_start", op.handle)
    return CgState(op, h, b3.shape[0])


def btoep_cg_state_size(op_lo, op_hi, k):
    """(device bytes, pinned host bytes) of a stepwise CG state for k right-hand sides."""
    dev, host = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().btoep_cg_state_size(op_lo.handle, op_hi.handle if op_hi is not None else None, int(k),
                                              ctypes.byref(dev), ctypes.byref(host)),
           "btoep_cg_state_size", op_lo.handle)
    return dev.value, host.value


def btoep_cg_begin(op_lo, op_hi, b, x, rtol, inner_rtol, dev_mem, host_mem, stream=None):
    """Stepwise CG on caller memory (no allocation, no synchronisation).

    b, x : [k][Nt][Nm], float64 with a refinement operator ``op_hi``, else op_lo's vector type.
    dev_mem : uint8 CUDA tensor, host_mem : pinned uint8 CPU tensor, at least
    btoep_cg_state_size bytes each; kept alive by the returned state."""
    torch = _torch()
    vt = torch.float64 if op_hi is not None else op_lo.vector_dtype
    b3 = _vec(op_lo, b, (op_lo.Nt, op_lo.Nm), "b", dtype=vt)
    x3 = _vec(op_lo, x, (op_lo.Nt, op_lo.Nm), "x", dtype=vt)
    if x3.shape != b3.shape:
        raise ValueError("x and b must have the same shape")
    if not dev_mem.is_cuda or not dev_mem.is_contiguous():
        raise ValueError("dev_mem must be a contiguous CUDA tensor")
    if host_mem.is_cuda or not host_mem.is_pinned():
        raise ValueError("host_mem must be pinned host memory")
    h = ctypes.c_void_p()
    _check(load_library().btoep_cg_begin(
        op_lo.handle, op_hi.handle if op_hi is not None else None, b3.shape[0], ctypes.c_void_p(b3.data_ptr()),
        ctypes.c_void_p(x3.data_ptr()), float(rtol), float(inner_rtol), ctypes.c_void_p(dev_mem.data_ptr()),
        dev_mem.numel() * dev_mem.element_size(), ctypes.c_void_p(host_mem.data_ptr()),
        host_mem.numel() * host_mem.element_size(), _stream(stream), ctypes.byref(h)), "btoep_cg_begin",
        op_lo.handle)
    return CgState(op_lo, h, b3.shape[0], op_hi=op_hi, keep=(dev_mem, host_mem, b, x))


def btoep_cg_refine(cg, stream=None):
    """After Hx = H_hi x: true residual in FP64, outer test, restart of the inner iteration."""
    _check(load_library().btoep_cg_refine(cg.handle, _stream(stream)), "btoep_cg_refine", cg.op.handle)


def btoep_cg_report(cg):
    """(ready, [per right-hand side dict]) of the last landed poll -- never blocks."""
    ready = ctypes.c_int()
    res = (CgResult * cg.k)()
    _check(load_library().btoep_cg_report(cg.handle, ctypes.byref(ready), res), "btoep_cg_report", cg.op.handle)
    if not ready.value:
        return False, None
    return True, [dict(inner_iters=r.inner_iters, outer_iters=r.outer_iters, matvecs=r.matvecs,
                       converged=bool(r.converged), rel_residual=r.rel_residual) for r in res]


def btoep_cg_workspace_size(op_lo, op_hi, k=1):
    """Workspace bytes of btoep_cg_solve(op_lo, op_hi, k)."""
    n = ctypes.c_size_t()
    _check(load_library().btoep_cg_workspace_size(op_lo.handle, op_hi.handle if op_hi is not None else None,
                                                  int(k), ctypes.byref(n)), "btoep_cg_workspace_size",
           op_lo.handle)
    return n.value


def btoep_cg_update(cg, stream=None):
    _check(load_library().btoep_cg_update(cg.handle, _stream(stream)), "btoep_cg_update", cg.op.handle)


def btoep_cg_poll(cg, stream=None):
    _check(load_library().btoep_cg_poll(cg.handle, _stream(stream)), "btoep_cg_poll", cg.op.handle)


def btoep_cg_status(cg):
    """(ready, active, iters, [rel residual per right-hand side]) -- never blocks."""
    ready, active, iters = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rel = (ctypes.c_double * cg.k)()
    _check(load_library().btoep_cg_status(cg.handle, ctypes.byref(ready), ctypes.byref(active),
                                          ctypes.byref(iters), rel), "btoep_cg_status", cg.op.handle)
    return bool(ready.value), active.value, iters.value, list(rel)


def btoep_cg_end(cg):
    cg.end()


def btoep_apply_batched_ptrs(op, which, in_ptrs, out_ptrs, noise_prec=1.0, prior_prec=1.0, ws=None, stream=None):
    """Pointer-array apply on raw device addresses (ints); see btoep_apply_batched."""
    k = len(in_ptrs)
    if k != len(out_ptrs) or k > MAX_BATCH:
        raise ValueError("need len(in_ptrs) == len(out_ptrs) <= %d" % MAX_BATCH)
    PA = ctypes.c_void_p * max(k, 1)
    wp, wn = _ws(ws)
    _check(load_library().btoep_apply_batched(op.handle, WHICH[which], k, PA(*in_ptrs), PA(*out_ptrs),
                                              float(noise_prec), float(prior_prec), wp, wn, _stream(stream)),
           "btoep_apply_batched", op.handle)


class ApplyGraph:
    """One apply of k right-hand sides captured into a HIP graph (btoep_graph_*).

    ``launch(in_ptrs, out_ptrs)`` points the replay at other vectors (device addresses, ints);
    without them it reuses the previous ones.  All launches of one graph must go to one
    stream (they share the graph's address table and the workspace).
    """

    def __init__(self, op, which, k, noise_prec=1.0, prior_prec=1.0, ws=None):
        torch = _torch()
        k = int(k)
        if not 1 <= k <= MAX_BATCH:
            raise ValueError("k must be in 1..%d" % MAX_BATCH)
        self.op, self.which, self.k = op, which, k
        if ws is None:
            ws = torch.empty(btoep_workspace_size(op, which, k), dtype=torch.uint8,
                             device=torch.device("cuda", op.info["device"]))
        self.ws = ws
        self.handle = None
        self._arr = ctypes.c_void_p * k
        h = ctypes.c_void_p()
        wp, wn = _ws(ws)
        _check(load_library().btoep_graph_create(op.handle, WHICH[which], k, float(noise_prec), float(prior_prec),
                                                 wp, wn, ctypes.byref(h)), "btoep_graph_create", op.handle)
        self.handle = h

    def launch(self, in_ptrs=None, out_ptrs=None, stream=None):
        if in_ptrs is None:
            pin = pout = None
        else:
            if len(in_ptrs) != self.k or len(out_ptrs) != self.k:
                raise ValueError("graph holds %d right-hand sides" % self.k)
            pin, pout = self._arr(*in_ptrs), self._arr(*out_ptrs)
        _check(load_library().btoep_graph_launch(self.handle, pin, pout, _stream(stream)), "btoep_graph_launch",
               self.op.handle)

    def destroy(self):
        if self.handle:
            load_library().btoep_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
