"""The appendix (SOTI) form of the local matvec against the oracle (needs an MI355X).

Both forms -- products written out and reduced separately (mode 0, as in the paper's
appendix) and products formed inside the reduction (mode 1) -- must give F m and F^T d to the
same tolerance as the main path, on ragged shapes, on a long series (four-step transforms),
on degenerate sizes and with many parameter chunks.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import make, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 3e-3}
SHAPES = [(37, 5, 301), (1, 1, 1), (9, 1, 40), (64, 12, 1), (5000, 3, 70)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("mode", [0, 1])
def test_alt_forms_match_the_oracle(bt, shape, storage, mode):
    Nt, Nd, Nm = shape
    print("alt", shape, storage, mode, flush=True)
    blocks = synth.blocks(Nt, Nd, Nm, tau=max(Nt / 6, 1.0), seed=101)
    op = make(bt, blocks, storage)
    bt.btoep_alt_prepare(op, mode)
    m = synth.vectors(1, Nt, Nm, stream=102)[0]
    d = synth.vectors(1, Nt, Nd, stream=103)[0]
    vt = op.vector_dtype
    got_F = bt.btoep_alt_apply(op, "F", to_dev(m, vt), mode=mode).double().cpu().numpy()
    got_FT = bt.btoep_alt_apply(op, "FT", to_dev(d, vt), mode=mode).double().cpu().numpy()
    assert oracle.rel_l2(got_F, oracle.apply_F(blocks, m)) <= TOL[storage]
    assert oracle.rel_l2(got_FT, oracle.apply_FT(blocks, d)) <= TOL[storage]
    # and the main path, to the same bar
    main_F = bt.btoep_apply_F(op, to_dev(m, vt)).double().cpu().numpy()
    assert oracle.rel_l2(got_F, main_F) <= 2 * TOL[storage]


@pytest.mark.parametrize("mode", [0, 1])
def test_alt_forms_with_many_parameter_chunks(bt, mode):
    """Nm large enough for several chunks of the sums over p; sampled oracle entries."""
    Nt, Nd, Nm = 420, 7, 40000
    blocks = synth.blocks(Nt, Nd, Nm, tau=60.0, seed=104)
    op = make(bt, blocks, "f32")
    bt.btoep_alt_prepare(op, mode)
    rng = np.random.default_rng(7)
    m = synth.vectors(1, Nt, Nm, stream=105)[0]
    d = synth.vectors(1, Nt, Nd, stream=106)[0]
    got_F = bt.btoep_alt_apply(op, "F", to_dev(m, torch.float32), mode=mode).double().cpu().numpy()
    got_FT = bt.btoep_alt_apply(op, "FT", to_dev(d, torch.float32), mode=mode).double().cpu().numpy()
    idx_F = [(int(i), int(s)) for i, s in zip(rng.integers(0, Nt, 48), rng.integers(0, Nd, 48))]
    idx_FT = [(int(j), int(p)) for j, p in zip(rng.integers(0, Nt, 48), rng.integers(0, Nm, 48))]
    ref_F = oracle.entries_F(blocks, m, idx_F)
    ref_FT = oracle.entries_FT(blocks, d, idx_FT)
    assert oracle.rel_l2([got_F[i, s] for i, s in idx_F], ref_F) <= 1e-5
    assert oracle.rel_l2([got_FT[j, p] for j, p in idx_FT], ref_FT) <= 1e-5


def test_alt_apply_requires_prepare(bt):
    import ctypes
    lib = bt.load_library()
    op = make(bt, synth.blocks(8, 2, 16, tau=4.0, seed=107), "f32")
    x = torch.zeros((8, 16), dtype=torch.float32, device="cuda")
    y = torch.zeros((8, 2), dtype=torch.float32, device="cuda")
    px, py = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    assert lib.btoep_alt_apply(op.handle, 0, 1, px, py, None) == 1  # not prepared
    assert lib.btoep_alt_prepare(op.handle, 1, None) == 0
    assert lib.btoep_alt_apply(op.handle, 0, 0, px, py, None) == 1  # product buffer not made
    assert lib.btoep_alt_apply(op.handle, 2, 1, px, py, None) == 1  # H is not offered
    assert lib.btoep_alt_prepare(op.handle, 2, None) == 1
    assert lib.btoep_alt_apply(op.handle, 0, 1, px, py, None) == 0
