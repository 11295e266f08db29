"""HIP path vs the FP64 oracle on seeded inputs, through the C-ABI (needs an MI355X).

Tolerances (relative l2 over the whole output): 1e-12 for an FP64-stored operator,
1e-5 for FP32, 3e-3 for BF16 (FP32 vectors and accumulation in both low precisions).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests import pins
from tests.gpu_helpers import gpu_F, gpu_FT, gpu_H, make, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 3e-3}


def run_all_three(bt, op, m, d, noise_prec=1.0, prior_prec=1.0):
    vt = op.vector_dtype
    Fm = bt.btoep_apply_F(op, to_dev(m, vt))
    FTd = bt.btoep_apply_FT(op, to_dev(d, vt))
    Hm = bt.btoep_apply_H(op, to_dev(m, vt), noise_prec, prior_prec)
    torch.cuda.synchronize()
    return [t.double().cpu().numpy() for t in (Fm, FTd, Hm)]


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_fp64_small_workload(bt, storage):
    """Nt=32, Nd=16, Nm=64, F_k = N(0,1) exp(-k/8); full output vectors."""
    w = synth.WORKLOADS["fp64-small"]
    print("case fp64-small", storage, flush=True)
    blocks = synth.blocks(w["Nt"], w["Nd"], w["Nm"], w["tau"])
    m = synth.vectors(1, w["Nt"], w["Nm"], synth.STREAM_M)[0]
    d = synth.vectors(1, w["Nt"], w["Nd"], synth.STREAM_D)[0]
    op = make(bt, blocks, storage)
    Fm, FTd, Hm = run_all_three(bt, op, m, d)
    assert oracle.rel_l2(Fm, oracle.apply_F(blocks, m)) <= TOL[storage]
    assert oracle.rel_l2(FTd, oracle.apply_FT(blocks, d)) <= TOL[storage]
    assert oracle.rel_l2(Hm, oracle.apply_H(blocks, m, 1.0, 1.0)) <= TOL[storage]


def test_every_pin_through_the_gpu_path(bt):
    """The oracle's pins (brute force, LTI time stepping, convolution, delta, closed form,
    adjoint, Hessian, shift, linearity) hold for the FP64 HIP path too."""
    errs = pins.run_all(gpu_F(bt, "f64"), gpu_FT(bt, "f64"), gpu_H(bt, "f64"))
    bad = {k: v for k, v in errs.items() if not v <= 1e-12}
    assert not bad, errs


# shapes: ragged Nm (not a multiple of 8 or of a span), Nd not a multiple of the row block,
# Nt whose transform length needs padding beyond 2 Nt (11 -> N 12), primes, several
# FFT column tiles and several spans
RAGGED = [(1, 1, 1), (2, 3, 5), (11, 5, 13), (13, 7, 1000), (37, 9, 300), (64, 100, 4099), (45, 3, 9001),
          (128, 50, 2000), (17, 130, 257)]


@pytest.mark.parametrize("shape", RAGGED)
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_ragged_shapes(bt, shape, storage):
    Nt, Nd, Nm = shape
    print("case ragged", shape, storage, flush=True)
    rng = np.random.default_rng(Nt * 1000 + Nd * 10 + Nm)
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / max(Nt / 7, 1))[:, None, None]
    m = rng.standard_normal((Nt, Nm))
    d = rng.standard_normal((Nt, Nd))
    op = make(bt, blocks, storage)
    Fm, FTd, Hm = run_all_three(bt, op, m, d, 2.0, 0.5)
    tol = TOL[storage]
    if storage == "bf16" and Nt * min(Nd, Nm) < 16:
        # a handful of terms per output: no averaging of the rounding errors, so use the
        # worst case of one BF16 rounding of the operator (unit roundoff u = 2^-8) entering
        # H twice: (1 + u)^2 - 1
        tol = (1 + 2.0 ** -8) ** 2 - 1
    assert oracle.rel_l2(Fm, oracle.apply_F(blocks, m)) <= tol
    assert oracle.rel_l2(FTd, oracle.apply_FT(blocks, d)) <= tol
    assert oracle.rel_l2(Hm, oracle.apply_H(blocks, m, 2.0, 0.5)) <= tol


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_multi_rhs_and_pointer_batches(bt, storage):
    """k right-hand sides stacked, and the pointer-array form, equal solo runs (bitwise)."""
    rng = np.random.default_rng(11)
    Nt, Nd, Nm, k = 24, 6, 700, 5
    blocks = rng.standard_normal((Nt, Nd, Nm))
    op = make(bt, blocks, storage)
    vt = op.vector_dtype
    M = to_dev(rng.standard_normal((k, Nt, Nm)), vt)
    D = to_dev(rng.standard_normal((k, Nt, Nd)), vt)
    FM = bt.btoep_apply_F(op, M)
    FTD = bt.btoep_apply_FT(op, D)
    HM = bt.btoep_apply_H(op, M, 3.0, 0.25)
    outs = [torch.empty((Nt, Nm), dtype=vt, device="cuda") for _ in range(k)]
    bt.btoep_apply_batched(op, "H", [M[r] for r in range(k)], outs, 3.0, 0.25)
    outs_f = [torch.empty((Nt, Nd), dtype=vt, device="cuda") for _ in range(k)]
    bt.btoep_apply_batched(op, "F", [M[r] for r in range(k)], outs_f)
    for r in range(k):
        assert torch.equal(bt.btoep_apply_F(op, M[r]), FM[r])
        assert torch.equal(bt.btoep_apply_FT(op, D[r]), FTD[r])
        assert torch.equal(bt.btoep_apply_H(op, M[r], 3.0, 0.25), HM[r])
        assert torch.equal(outs[r], HM[r])
        assert torch.equal(outs_f[r], FM[r])
    Mn = M.double().cpu().numpy()
    assert oracle.rel_l2(FM.double().cpu().numpy(), oracle.apply_F(blocks, Mn)) <= TOL[storage]


def test_repeat_calls_are_bitwise_identical(bt):
    rng = np.random.default_rng(12)
    blocks = rng.standard_normal((40, 10, 5000))
    op = make(bt, blocks, "f32")
    m = to_dev(rng.standard_normal((40, 5000)), torch.float32)
    a = bt.btoep_apply_H(op, m, 1.0, 1.0)
    b = bt.btoep_apply_H(op, m, 1.0, 1.0)
    assert torch.equal(a, b)


def test_device_resident_blocks_match_host_blocks(bt):
    rng = np.random.default_rng(13)
    blocks = rng.standard_normal((20, 4, 333))
    op_h = make(bt, blocks, "f32")
    op_d = bt.btoep_create(torch.from_numpy(blocks).cuda(), "f32")
    m = to_dev(rng.standard_normal((20, 333)), torch.float32)
    assert torch.equal(bt.btoep_apply_F(op_h, m), bt.btoep_apply_F(op_d, m))


def test_query_and_workspace(bt):
    blocks = np.ones((420, 3, 17))
    op = make(bt, blocks, "bf16")
    info = bt.btoep_query(op)
    assert info["L"] == 840 and info["nfreq"] == 421 and info["ldF"] == 24
    assert info["fhat_bytes"] == 421 * 3 * 24 * 4
    assert bt.btoep_workspace_size(op, "H", 4) > bt.btoep_workspace_size(op, "H", 1) > 0
    ws = torch.empty(bt.btoep_workspace_size(op, "F", 1) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(bt.BtoepError):
        bt.btoep_apply_F(op, torch.zeros((420, 17), dtype=torch.float32, device="cuda"), ws=ws)


def test_unsupported_length_is_an_error(bt):
    with pytest.raises(bt.BtoepError):
        bt.btoep_create(np.zeros((5000, 1, 1)), "f64")
