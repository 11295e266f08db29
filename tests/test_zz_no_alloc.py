"""btoep_apply_static (the applies with the library's static device scratch as workspace, for
callers that cannot allocate) against btoep_apply_F / _FT / _H with a caller workspace: the
same launches, so the results are bitwise equal; two calls in a row, the second with fewer
right-hand sides (what the first left in the shared scratch must not matter), in every
storage; and a request whose workspace exceeds the scratch is refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from tests.gpu_helpers import make

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("which", ["F", "FT", "H"])
def test_static_scratch_apply_equals_workspace_apply(bt, storage, which):
    Nt, Nd, Nm = 37, 5, 300
    print("case static apply", storage, which, flush=True)
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 7.0, seed=91)
    op = make(bt, blocks, storage)
    n_in = Nd if which == "FT" else Nm
    n_out = Nd if which == "F" else Nm
    gen = torch.Generator(device="cuda").manual_seed(91)
    for k in (9, 3):   # second call smaller than the first
        x = torch.randn((k, Nt, n_in), generator=gen, device="cuda", dtype=op.vector_dtype)
        got = torch.full((k, Nt, n_out), float("nan"), device="cuda", dtype=op.vector_dtype)
        bt.btoep_apply_static(op, which, x, got, noise_prec=2.0, prior_prec=0.5)
        ws = torch.empty(bt.btoep_workspace_size(op, which, k), dtype=torch.uint8, device="cuda")
        if which == "F":
            want = bt.btoep_apply_F(op, x, ws=ws)
        elif which == "FT":
            want = bt.btoep_apply_FT(op, x, ws=ws)
        else:
            want = bt.btoep_apply_H(op, x, 2.0, 0.5, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (storage, which, k)
    op.destroy()


def test_static_scratch_refuses_oversized_applies(bt):
    Nt, Nd, Nm = 420, 4, 65536   # the spectra of one right-hand side alone exceed 128 MiB
    blocks = np.zeros((Nt, Nd, Nm))
    op = bt.btoep_create(blocks, "f32")
    assert bt.btoep_workspace_size(op, "H", 1) > bt.STATIC_SCRATCH_BYTES
    x = torch.zeros((1, Nt, Nm), device="cuda")
    out = torch.full_like(x, 7.0)
    lib = bt.load_library()
    st = lib.btoep_apply_static(op.handle, 2, 1, 1.0, 1.0, ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), None)
    torch.cuda.synchronize()
    assert st == bt.BTOEP_ERR_WORKSPACE_TOO_SMALL
    assert b"static scratch" in lib.btoep_last_error(op.handle)
    assert bool((out == 7.0).all())   # nothing was launched
    op.destroy()
