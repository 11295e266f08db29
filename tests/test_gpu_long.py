"""Four-step transforms for long time series (N = N1 N2) through the C-ABI (needs an MI355X).

The four-step path computes the same length-2N DFTs as the single-pass kernels, so every
apply must match the FP64 oracle at the storage tolerance whichever factorisation is used,
forced on ordinary shapes and chosen automatically when a series does not fit one
workgroup's LDS.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import make, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 3e-3}


def apply_all(bt, op, m, d, noise, prior):
    vt = op.vector_dtype
    M, D = to_dev(m, vt), to_dev(d, vt)
    out = (bt.btoep_apply_F(op, M), bt.btoep_apply_FT(op, D), bt.btoep_apply_H(op, M, noise, prior))
    torch.cuda.synchronize()
    return [o.double().cpu().numpy() for o in out]


def check(bt, blocks, storage, k, n1, seed, noise=2.0, prior=0.5):
    Nt, Nd, Nm = blocks.shape
    m = synth.vectors(k, Nt, Nm, stream=60 + seed)
    d = synth.vectors(k, Nt, Nd, stream=70 + seed)
    refs = (oracle.apply_F(blocks, m), oracle.apply_FT(blocks, d), oracle.apply_H(blocks, m, noise, prior))
    op = make(bt, blocks, storage)
    single = apply_all(bt, op, m, d, noise, prior)
    bt.btoep_set_fft(op, n1)
    four = apply_all(bt, op, m, d, noise, prior)
    tol = TOL[storage]
    for name, ref, a, b in zip(("F", "FT", "H"), refs, single, four):
        assert oracle.rel_l2(b, ref) <= tol, (name, storage, n1, oracle.rel_l2(b, ref))
        assert oracle.rel_l2(b, a) <= 2 * tol, (name, storage, n1)


# (Nt, Nd, Nm), k, n1: N = Nt (7-smooth) split as n1 x N/n1; ragged Nm and Nd, several tiles
FORCED = [((32, 5, 300), 1, 4), ((32, 5, 300), 3, 8), ((60, 7, 1000), 2, 6), ((105, 3, 257), 1, 7),
          ((128, 9, 700), 8, 16), ((420, 4, 130), 1, 20), ((420, 4, 130), 5, 21), ((48, 2, 33), 17, 6),
          # sub-transforms with compile-time plans (100 x 100, 50 x 100, 100 x 50)
          ((10000, 2, 37), 1, 100), ((5000, 3, 70), 2, 50), ((5000, 3, 70), 1, 100)]


@pytest.mark.parametrize("shape,k,n1", FORCED)
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_forced_four_step_matches_oracle(bt, shape, k, n1, storage):
    Nt, Nd, Nm = shape
    print("four-step case", shape, k, n1, storage, flush=True)
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 6.0, seed=91)
    check(bt, blocks, storage, k, n1, seed=k)


def test_invalid_factor_keeps_a_working_operator(bt):
    blocks = synth.blocks(30, 3, 50, tau=5.0, seed=92)
    op = make(bt, blocks, "f32")
    with pytest.raises(bt.BtoepError):
        bt.btoep_set_fft(op, 7)  # 7 does not divide N = 30
    m = synth.vectors(1, 30, 50, stream=80)
    got = bt.btoep_apply_F(op, to_dev(m, torch.float32))
    torch.cuda.synchronize()
    assert oracle.rel_l2(got.double().cpu().numpy(), oracle.apply_F(blocks, m)) <= 1e-5


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_series_too_long_for_one_workgroup(bt, storage):
    """Nt = 4200: a length-N FP64 column does not fit one workgroup's LDS, so setup and applies
    switch to four-step transforms by themselves."""
    Nt, Nd, Nm = 4200, 3, 37
    print("long series", Nt, storage, flush=True)
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 7.0, seed=93)
    m = synth.vectors(2, Nt, Nm, stream=81)
    d = synth.vectors(2, Nt, Nd, stream=82)
    op = make(bt, blocks, storage)
    got = apply_all(bt, op, m, d, 3.0, 0.25)
    refs = (oracle.apply_F(blocks, m), oracle.apply_FT(blocks, d), oracle.apply_H(blocks, m, 3.0, 0.25))
    for name, ref, g in zip(("F", "FT", "H"), refs, got):
        assert oracle.rel_l2(g, ref) <= TOL[storage], (name, oracle.rel_l2(g, ref))
    with pytest.raises(bt.BtoepError):
        bt.btoep_set_fft(op, -1)  # single-pass does not fit: refused, four-step kept
    got2 = apply_all(bt, op, m, d, 3.0, 0.25)
    assert oracle.rel_l2(got2[0], refs[0]) <= TOL[storage]
