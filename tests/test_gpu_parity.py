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

TOL = {"f64": 1e-12, "f32": 1e-5, "f32split": 1e-5, "bf16": 3e-3}


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
# FFT column tiles and several spans, and every transform length with a compile-time plan
# (N = 32, 64, 128, 256, 420, 512) next to runtime-plan lengths
RAGGED = [(1, 1, 1), (2, 3, 5), (11, 5, 13), (13, 7, 1000), (37, 9, 300), (64, 100, 4099), (45, 3, 9001),
          (128, 50, 2000), (17, 130, 257), (512, 3, 700), (256, 12, 333), (420, 5, 1111),
          # lengths with compile-time FP64 plans (setup of every storage, FP64 vector transforms)
          (1000, 2, 129), (2000, 3, 77), (4000, 2, 37)]


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


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_multi_rhs_and_pointer_batches(bt, storage):
    """k right-hand sides stacked equal the pointer-array form bitwise, and solo runs (the
    single-vector kernels) within the tolerance."""
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
    outs_t = [torch.empty((Nt, Nm), dtype=vt, device="cuda") for _ in range(k)]
    bt.btoep_apply_batched(op, "FT", [D[r] for r in range(k)], outs_t)
    tol = TOL[storage]
    for r in range(k):
        assert torch.equal(outs[r], HM[r])
        assert torch.equal(outs_f[r], FM[r])
        assert torch.equal(outs_t[r], FTD[r])
        solo = [bt.btoep_apply_F(op, M[r]), bt.btoep_apply_FT(op, D[r]), bt.btoep_apply_H(op, M[r], 3.0, 0.25)]
        for a, b in zip(solo, (FM[r], FTD[r], HM[r])):
            assert oracle.rel_l2(a.double().cpu().numpy(), b.double().cpu().numpy()) <= tol
    Mn = M.double().cpu().numpy()
    Dn = D.double().cpu().numpy()
    FM_ref = oracle.apply_F(blocks, Mn)
    FTD_ref = oracle.apply_FT(blocks, Dn)
    HM_ref = oracle.apply_H(blocks, Mn, 3.0, 0.25)
    for r in range(k):
        assert oracle.rel_l2(FM[r].double().cpu().numpy(), FM_ref[r]) <= tol
        assert oracle.rel_l2(FTD[r].double().cpu().numpy(), FTD_ref[r]) <= tol
        assert oracle.rel_l2(HM[r].double().cpu().numpy(), HM_ref[r]) <= tol


# k crossing every tile width of the matrix-core kernels (8 right-hand sides per tile),
# with ragged Nm, Nd above one 128-row group, and Nd large enough that the adjoint's staged
# data spectra are split into groups
MULTI = [((13, 7, 1000), 2), ((13, 7, 1000), 9), ((64, 100, 4099), 8), ((64, 100, 4099), 17),
         ((17, 130, 257), 33), ((20, 200, 700), 64), ((9, 3, 130), 64)]


@pytest.mark.parametrize("shape,k", MULTI)
@pytest.mark.parametrize("storage", ["f64", "f32", "f32split", "bf16"])
def test_multi_rhs_matrix_cores(bt, shape, k, storage):
    Nt, Nd, Nm = shape
    print("case multi", shape, k, storage, flush=True)
    rng = np.random.default_rng(Nt + 7 * Nd + Nm + k)
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / max(Nt / 7, 1))[:, None, None]
    op = make(bt, blocks, storage)
    vn = np.float64 if storage == "f64" else np.float32
    M = rng.standard_normal((k, Nt, Nm)).astype(vn)
    D = rng.standard_normal((k, Nt, Nd)).astype(vn)
    Md, Dd = to_dev(M, op.vector_dtype), to_dev(D, op.vector_dtype)
    FM = bt.btoep_apply_F(op, Md).double().cpu().numpy()
    FTD = bt.btoep_apply_FT(op, Dd).double().cpu().numpy()
    HM = bt.btoep_apply_H(op, Md, 1.5, 0.75).double().cpu().numpy()
    M64, D64 = M.astype(np.float64), D.astype(np.float64)
    FM_ref = oracle.apply_F(blocks, M64)
    FTD_ref = oracle.apply_FT(blocks, D64)
    HM_ref = oracle.apply_H(blocks, M64, 1.5, 0.75)
    tol = TOL[storage]
    for r in range(k):
        assert oracle.rel_l2(FM[r], FM_ref[r]) <= tol, ("F", r)
        assert oracle.rel_l2(FTD[r], FTD_ref[r]) <= tol, ("FT", r)
        assert oracle.rel_l2(HM[r], HM_ref[r]) <= tol, ("H", r)


# FP64 series lengths with compile-time plans, one and several vectors: the launchers pick the
# fused or the general transform kernels by tile width and vector count, so both meet here
# (N = 420: 8-column tiles, N = 1000: 4, N = 2000: 2), with ragged column tiles.
@pytest.mark.parametrize("shape", [(420, 3, 1111), (1000, 2, 129), (2000, 3, 77)])
@pytest.mark.parametrize("k", [1, 3])
def test_fp64_transforms_by_vector_count(bt, shape, k):
    Nt, Nd, Nm = shape
    print("case fp64 transforms", shape, k, flush=True)
    rng = np.random.default_rng(Nt + Nd + Nm + 100 * k)
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / (Nt / 7))[:, None, None]
    op = make(bt, blocks, "f64")
    M = rng.standard_normal((k, Nt, Nm))
    D = rng.standard_normal((k, Nt, Nd))
    Md, Dd = to_dev(M, torch.float64), to_dev(D, torch.float64)
    FM = bt.btoep_apply_F(op, Md).cpu().numpy()
    FTD = bt.btoep_apply_FT(op, Dd).cpu().numpy()
    HM = bt.btoep_apply_H(op, Md, 2.0, 0.5).cpu().numpy()
    FM_ref = oracle.apply_F(blocks, M)
    FTD_ref = oracle.apply_FT(blocks, D)
    HM_ref = oracle.apply_H(blocks, M, 2.0, 0.5)
    for r in range(k):
        assert oracle.rel_l2(FM[r], FM_ref[r]) <= TOL["f64"], ("F", r)
        assert oracle.rel_l2(FTD[r], FTD_ref[r]) <= TOL["f64"], ("FT", r)
        assert oracle.rel_l2(HM[r], HM_ref[r]) <= TOL["f64"], ("H", r)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("storage", ["f32", "f32split", "bf16"])
def test_multi_rhs_on_a_wide_launch(bt, storage):
    """Enough (span, frequency) workgroups (66 x 65) for the forward product's wide chunks of
    vector columns, with a ragged last span (Nm = 65 x 4096 + 3761)."""
    Nt, Nd, Nm, k = 64, 3, 270001, 8
    print("wide multi", storage, flush=True)
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 6, seed=111)
    op = make(bt, blocks, storage)
    M = synth.vectors(k, Nt, Nm, stream=112)
    Md = to_dev(M, op.vector_dtype)
    M64 = Md.double().cpu().numpy()  # the vectors as the device holds them
    FM = bt.btoep_apply_F(op, Md).double().cpu().numpy()
    HM = bt.btoep_apply_H(op, Md, 1.5, 0.75).double().cpu().numpy()
    FM_ref = oracle.apply_F(blocks, M64)
    HM_ref = oracle.apply_H(blocks, M64[[0, 5]], 1.5, 0.75)
    tol = TOL[storage]
    for r in range(k):
        assert oracle.rel_l2(FM[r], FM_ref[r]) <= tol, ("F", r)
    for i, r in enumerate((0, 5)):
        assert oracle.rel_l2(HM[r], HM_ref[i]) <= tol, ("H", r)


@pytest.mark.parametrize("storage", ["f64", "f32", "f32split", "bf16"])
def test_matrix_core_results_are_batch_invariant(bt, storage):
    """A right-hand side gives bitwise the same result in any batch of k >= 2 and at any position."""
    rng = np.random.default_rng(41)
    Nt, Nd, Nm = 30, 20, 1500
    op = make(bt, rng.standard_normal((Nt, Nd, Nm)), storage)
    V = to_dev(rng.standard_normal((12, Nt, Nm)), op.vector_dtype)
    big = bt.btoep_apply_H(op, V, 2.0, 0.5)
    small = bt.btoep_apply_H(op, V[[7, 3, 9]].contiguous(), 2.0, 0.5)
    for a, b in zip((7, 3, 9), range(3)):
        assert torch.equal(big[a], small[b])
    Fb = bt.btoep_apply_F(op, V)
    Fs = bt.btoep_apply_F(op, V[[11, 0]].contiguous())
    assert torch.equal(Fb[11], Fs[0]) and torch.equal(Fb[0], Fs[1])


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


@pytest.mark.parametrize("Nt", [5000, 64827])
def test_long_series_supported_and_overlong_refused(bt, Nt):
    """Nt = 5000 does not fit one workgroup in FP64 (four-step transforms take over); Nt = 64827
    is the longest series (65535 stored frequencies, the products' grid limit), checked against
    np.convolve for F and np.correlate for F^T; one step more and create refuses."""
    rng = np.random.default_rng(9)
    blocks = rng.standard_normal((Nt, 1, 1)) * np.exp(-np.arange(Nt) / (Nt / 7.0))[:, None, None]
    m = rng.standard_normal((Nt, 1))
    print("long series", Nt, flush=True)
    op = bt.btoep_create(blocks, "f64")
    assert op.info["nfreq"] <= 65535
    d = bt.btoep_apply_F(op, to_dev(m, torch.float64))
    mt = bt.btoep_apply_FT(op, to_dev(m, torch.float64))
    torch.cuda.synchronize()
    ref = np.convolve(blocks[:, 0, 0], m[:, 0])[:Nt]
    assert oracle.rel_l2(d.cpu().numpy()[:, 0], ref) <= 1e-12
    # (F^T d)_j = sum_{i >= j} F_{i-j} d_i: the correlation of d with the block sequence
    ref_t = np.correlate(m[:, 0], blocks[:, 0, 0], mode="full")[Nt - 1:]
    assert oracle.rel_l2(mt.cpu().numpy()[:, 0], ref_t) <= 1e-12
    if Nt == 64827:
        with pytest.raises(bt.BtoepError) as e:
            bt.btoep_create(np.zeros((Nt + 1, 1, 1)), "f64")
        assert e.value.status == 4


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_every_kernel_variant_and_autotune(bt, storage):
    """Each tuning variant of the single-vector products, and the per-vector path for several
    right-hand sides, matches the oracle; autotune returns a valid choice."""
    rng = np.random.default_rng(51)
    Nt, Nd, Nm = 23, 19, 4099 + 512
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / 4.0)[:, None, None]
    op = make(bt, blocks, storage)
    m = rng.standard_normal((2, Nt, Nm))
    d = rng.standard_normal((2, Nt, Nd))
    vt = op.vector_dtype
    Fm_ref, FTd_ref = oracle.apply_F(blocks, m), oracle.apply_FT(blocks, d)
    for var in range(6):
        for mfma in (True, False):
            bt.btoep_set_tuning(op, var, var, mfma)
            Fm = bt.btoep_apply_F(op, to_dev(m, vt)).double().cpu().numpy()
            FTd = bt.btoep_apply_FT(op, to_dev(d, vt)).double().cpu().numpy()
            for r in range(2):
                assert oracle.rel_l2(Fm[r], Fm_ref[r]) <= TOL[storage], (var, mfma)
                assert oracle.rel_l2(FTd[r], FTd_ref[r]) <= TOL[storage], (var, mfma)
    t = bt.btoep_autotune(op, reps=2)
    assert 0 <= t["var_n"] < 6 and 0 <= t["var_c"] < 6 and len(t["ms_n"]) == 6
    with pytest.raises(bt.BtoepError):
        bt.btoep_set_tuning(op, 6, 0)


@pytest.mark.parametrize("shape", [(5, 65535, 9), (3, 2, 1000003)])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 3])
def test_extreme_sensor_and_parameter_counts(bt, shape, storage, k):
    """The largest sensor count the library accepts (65535: a grid dimension of the data-side
    kernel) and a million ragged parameter columns, single- and multi-vector."""
    Nt, Nd, Nm = shape
    print("extreme", shape, storage, k, flush=True)
    rng = np.random.default_rng(Nd + Nm + k)
    blocks = rng.standard_normal((Nt, Nd, Nm))
    op = make(bt, blocks, storage)
    vn = np.float64 if storage == "f64" else np.float32
    M = rng.standard_normal((k, Nt, Nm)).astype(vn)
    D = rng.standard_normal((k, Nt, Nd)).astype(vn)
    FM = bt.btoep_apply_F(op, to_dev(M, op.vector_dtype)).double().cpu().numpy()
    FTD = bt.btoep_apply_FT(op, to_dev(D, op.vector_dtype)).double().cpu().numpy()
    FM_ref = oracle.apply_F(blocks, M.astype(np.float64))
    FTD_ref = oracle.apply_FT(blocks, D.astype(np.float64))
    for r in range(k):
        assert oracle.rel_l2(FM[r], FM_ref[r]) <= TOL[storage]
        assert oracle.rel_l2(FTD[r], FTD_ref[r]) <= TOL[storage]
    with pytest.raises(bt.BtoepError) as e:
        bt.btoep_create(np.zeros((2, 65536, 1)), storage)
    assert e.value.status == 4


@pytest.mark.parametrize("storage", ["f32split", "bf16"])
def test_adjoint_products_staged_in_phases(bt, storage):
    """BF16 / split adjoint products stage the data spectra in phases of at most 64 sensors (eight
    tiles) or 128 (four tiles): Nd = 150 takes three and two phases, with a ragged last one, in every
    adjoint variant; F^T and H against the oracle."""
    rng = np.random.default_rng(83)
    Nt, Nd, Nm = 9, 150, 700
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / 3.0)[:, None, None]
    op = make(bt, blocks, storage)
    tol = TOL[storage]
    for k in (20, 40):
        print("case adjoint phases", storage, k, flush=True)
        D = rng.standard_normal((k, Nt, Nd)).astype(np.float32)
        M = rng.standard_normal((k, Nt, Nm)).astype(np.float32)
        FTD_ref = oracle.apply_FT(blocks, D.astype(np.float64))
        HM_ref = oracle.apply_H(blocks, M[[0, k - 1]].astype(np.float64), 2.0, 0.5)
        for var_c in range(N_GEMM_C_VARIANTS):
            bt.btoep_set_gemm_variants(op, k, 0, var_c)
            FTD = bt.btoep_apply_FT(op, to_dev(D, torch.float32)).double().cpu().numpy()
            for r in range(k):
                assert oracle.rel_l2(FTD[r], FTD_ref[r]) <= tol, ("FT", k, var_c, r)
            HM = bt.btoep_apply_H(op, to_dev(M, torch.float32), 2.0, 0.5)[[0, k - 1]].double().cpu().numpy()
            for i in range(2):
                assert oracle.rel_l2(HM[i], HM_ref[i]) <= tol, ("H", k, var_c, i)
    op.destroy()


# matrix-core kernel variants the library offers (forward, adjoint)
N_GEMM_N_VARIANTS, N_GEMM_C_VARIANTS = 5, 5


@pytest.mark.parametrize("storage", ["f32", "f32split", "bf16"])
def test_every_matrix_core_variant_and_gemm_autotune(bt, storage):
    """Every forward and adjoint matrix-core kernel variant, in every right-hand-side bucket
    (k = 9, 33 and 64 with ragged tiles; Nd past one 16-row tile group, ragged Nm), against the
    oracle; then the matrix-core autotuner's choice."""
    rng = np.random.default_rng(81)
    Nt, Nd, Nm = 11, 37, 1300
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / 3.0)[:, None, None]
    op = make(bt, blocks, storage)
    tol = TOL[storage]
    for k in (9, 33, 64):
        print("case gemm variants", storage, k, flush=True)
        M = rng.standard_normal((k, Nt, Nm)).astype(np.float32)
        D = rng.standard_normal((k, Nt, Nd)).astype(np.float32)
        Md, Dd = to_dev(M, torch.float32), to_dev(D, torch.float32)
        FM_ref = oracle.apply_F(blocks, M.astype(np.float64))
        FTD_ref = oracle.apply_FT(blocks, D.astype(np.float64))
        combos = [(v, 0) for v in range(N_GEMM_N_VARIANTS)] + [(0, v) for v in range(1, N_GEMM_C_VARIANTS)]
        for var_n, var_c in combos:
            bt.btoep_set_gemm_variants(op, k, var_n, var_c)
            FM = bt.btoep_apply_F(op, Md).double().cpu().numpy()
            FTD = bt.btoep_apply_FT(op, Dd).double().cpu().numpy()
            for r in range(k):
                assert oracle.rel_l2(FM[r], FM_ref[r]) <= tol, ("F", k, var_n, r)
                assert oracle.rel_l2(FTD[r], FTD_ref[r]) <= tol, ("FT", k, var_c, r)
        tune = bt.btoep_autotune_gemm(op, k, allow_split=(storage == "f32split"), reps=2)
        assert tune["nvar_n"] == N_GEMM_N_VARIANTS and tune["nvar_c"] == N_GEMM_C_VARIANTS
        assert 0 <= tune["var_n"] < N_GEMM_N_VARIANTS and 0 <= tune["var_c"] < N_GEMM_C_VARIANTS
        HM = bt.btoep_apply_H(op, Md, 1.5, 0.75).double().cpu().numpy()
        HM_ref = oracle.apply_H(blocks, M[:3].astype(np.float64), 1.5, 0.75)
        for r in range(3):
            assert oracle.rel_l2(HM[r], HM_ref[r]) <= tol, ("H after autotune", k, tune)
    with pytest.raises(bt.BtoepError):
        bt.btoep_set_gemm_variants(op, 9, N_GEMM_N_VARIANTS, 0)   # no such forward variant
    with pytest.raises(bt.BtoepError):
        bt.btoep_set_gemm_variants(op, 9, 0, N_GEMM_C_VARIANTS)   # no such adjoint variant
    with pytest.raises(bt.BtoepError):
        bt.btoep_set_gemm_variants(op, 1, 0, 0)   # one right-hand side has no matrix-core product
