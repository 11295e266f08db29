"""CG on H x = b through the C-ABI (needs an MI355X).

Pins: the dense solve of the assembled H on a tiny problem; the true residual recomputed by
the FP64 oracle's H; the same solution from plain FP64 CG and from low-precision inner CG
with FP64 iterative refinement.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests import pins
from tests.gpu_helpers import make, stepwise_cg, to_dev

pytestmark = pytest.mark.gpu


def solve(bt, lo, hi, b, noise_prec, prior_prec, **kw):
    bd = to_dev(b, torch.float64)
    x = torch.zeros_like(bd)
    st, res = bt.btoep_cg_solve(lo, hi, bd, x, noise_prec, prior_prec, **kw)
    torch.cuda.synchronize()
    return st, res, x.cpu().numpy()


def test_cg_tiny_matches_dense_solve(bt):
    rng = np.random.default_rng(21)
    Nt, Nd, Nm = 6, 2, 5
    blocks = rng.standard_normal((Nt, Nd, Nm))
    b = rng.standard_normal((Nt, Nm))
    noise_prec, prior_prec = 4.0, 0.1
    A = pins.dense_matrix(blocks)
    Hd = noise_prec * A.T @ A + prior_prec * np.eye(A.shape[1])
    x_ref = np.linalg.solve(Hd, b.ravel()).reshape(Nt, Nm)
    op = make(bt, blocks, "f64")
    st, res, x = solve(bt, op, None, b[None], noise_prec, prior_prec, rtol=1e-13, inner_rtol=1e-14,
                       max_inner=200)
    assert st == 0 and res[0]["converged"], res
    assert res[0]["rel_residual"] <= 1e-13
    assert oracle.rel_l2(x[0], x_ref) <= 1e-10


# Refinement contracts when the low-precision operator's perturbation of H, seen through
# the smallest eigenvalue prior_prec, stays below one: roughly eps^2 * lambda_max / prior_prec < 1
# with eps the relative error of the stored operator (FP32 ~3e-8, BF16 ~2e-3) and
# lambda_max ~ noise_prec * ||F||^2.  The FP32 case uses the inverse-problem scalars
# (sigma = 1e-2, alpha = 1e-3, lambda_max / alpha ~ 1e10); BF16 needs a milder prior.
@pytest.mark.parametrize("lo_storage,sigma,alpha,inner_rtol", [("f32", 1e-2, 1e-3, 1e-5),
                                                                ("bf16", 1.0, 10.0, 1e-2)])
def test_refinement_reaches_fp64_accuracy(bt, lo_storage, sigma, alpha, inner_rtol):
    """Low-precision inner CG inside FP64 refinement meets 1e-8 on the true residual and
    agrees with all-FP64 CG; checked with the oracle's H."""
    rng = np.random.default_rng(22)
    Nt, Nd, Nm, k = 48, 6, 700, 2
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / (Nt / 7))[:, None, None]
    m_true = rng.standard_normal((k, Nt, Nm))
    dobs = oracle.apply_F(blocks, m_true) + sigma * rng.standard_normal((k, Nt, Nd))
    noise_prec = sigma ** -2
    b = noise_prec * oracle.apply_FT(blocks, dobs)
    hi = make(bt, blocks, "f64")
    lo = make(bt, blocks, lo_storage)
    st, res, x = solve(bt, lo, hi, b, noise_prec, alpha, rtol=1e-8, inner_rtol=inner_rtol)
    print(lo_storage, res, flush=True)
    assert st == 0, res
    st64, res64, x64 = solve(bt, hi, None, b, noise_prec, alpha, rtol=1e-8, inner_rtol=1e-9)
    assert st64 == 0, res64
    for r in range(k):
        Hx = oracle.apply_H(blocks, x[r], noise_prec, alpha)
        assert np.linalg.norm(b[r] - Hx) / np.linalg.norm(b[r]) <= 1.01e-8
        Hx64 = oracle.apply_H(blocks, x64[r], noise_prec, alpha)
        assert np.linalg.norm(b[r] - Hx64) / np.linalg.norm(b[r]) <= 1.01e-8
        # data-space agreement of the two solutions (null-space components are not controlled)
        Fd = oracle.apply_F(blocks, x[r] - x64[r])
        assert np.linalg.norm(Fd) <= 1e-6 * np.linalg.norm(oracle.apply_F(blocks, x64[r]))


def test_cg_reports_not_converged(bt):
    rng = np.random.default_rng(23)
    blocks = rng.standard_normal((16, 4, 64))
    b = rng.standard_normal((1, 16, 64))
    op = make(bt, blocks, "f64")
    st, res, x = solve(bt, op, None, b, 1e4, 1e-3, rtol=1e-14, max_outer=1, max_inner=2, inner_rtol=1e-14)
    assert st == bt.BTOEP_ERR_NOT_CONVERGED
    assert not res[0]["converged"] and res[0]["rel_residual"] > 1e-14


def test_cg_inputs_validated(bt):
    blocks = np.ones((8, 2, 3))
    lo = make(bt, blocks, "f32")
    b = torch.zeros((1, 8, 3), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(bt.BtoepError):
        bt.btoep_cg_solve(lo, None, b, x, 1.0, 1.0)   # an FP32 operator needs an FP64 partner
    other = make(bt, np.ones((8, 2, 4)), "f64")
    with pytest.raises(bt.BtoepError):
        bt.btoep_cg_solve(lo, other, b, x, 1.0, 1.0)  # shapes differ


@pytest.mark.timeout(900)
def test_cg_workload_nt256_nd64_nm16384(bt):
    """H = sigma^-2 F^T F + alpha I, sigma = 1e-2, alpha = 1e-3, Nt=256, Nd=64, Nm=16384,
    d = F m_true + N(0, sigma^2), b = sigma^-2 F^T d: FP32 inner CG with FP64 refinement
    and plain FP64 CG both reach 1e-8, checked with the oracle's H."""
    w = synth.WORKLOADS["cg-nt256-nd64-nm16384"]
    Nt, Nd, Nm, tau = w["Nt"], w["Nd"], w["Nm"], w["tau"]
    print("case cg workload", flush=True)
    blocks = synth.blocks(Nt, Nd, Nm, tau)
    m_true = synth.vectors(1, Nt, Nm, synth.STREAM_MTRUE)[0]
    noise = synth.vectors(1, Nt, Nd, synth.STREAM_NOISE)[0]
    sigma, alpha = w["sigma"], w["alpha"]
    dobs = oracle.apply_F(blocks, m_true) + sigma * noise
    noise_prec = sigma ** -2
    b = noise_prec * oracle.apply_FT(blocks, dobs)
    hi = make(bt, blocks, "f64")
    lo = make(bt, blocks, "f32")
    st, res, x = solve(bt, lo, hi, b[None], noise_prec, alpha, rtol=w["rtol"], inner_rtol=1e-5)
    print("refined f32:", res, flush=True)
    assert st == 0
    st64, res64, x64 = solve(bt, hi, None, b[None], noise_prec, alpha, rtol=w["rtol"], inner_rtol=1e-9)
    print("fp64:", res64, flush=True)
    assert st64 == 0
    for xx in (x[0], x64[0]):
        Hx = oracle.apply_H(blocks, xx, noise_prec, alpha)
        assert np.linalg.norm(b - Hx) / np.linalg.norm(b) <= 1.01e-8


def test_stepwise_cg_with_a_caller_applied_prior(bt):
    """H with a general SPD prior R (here delta I + gamma times a path Laplacian over the
    parameters, at every time step): the caller runs the library's H at prior_prec = 0 and adds
    R p itself between the stepwise CG calls; the solution matches a dense solve of
    (noise_prec A^T A + R) x = b with A the assembled operator."""
    rng = np.random.default_rng(24)
    Nt, Nd, Nm = 6, 3, 8
    blocks = rng.standard_normal((Nt, Nd, Nm))
    noise_prec, delta, gamma = 2.0, 0.3, 0.7
    Rp = delta * np.eye(Nm) + gamma * (2 * np.eye(Nm) - np.eye(Nm, k=1) - np.eye(Nm, k=-1))
    A = pins.dense_matrix(blocks)
    Hd = noise_prec * A.T @ A + np.kron(np.eye(Nt), Rp)
    b = rng.standard_normal((1, Nt, Nm))
    x_ref = np.linalg.solve(Hd, b.ravel()).reshape(Nt, Nm)
    op = make(bt, blocks, "f64")
    bd = to_dev(b, torch.float64)
    x = torch.zeros_like(bd)
    cg = bt.btoep_cg_start(op, bd, x, 1e-12, noise_prec, 0.0)
    P, AP = cg.tensors()
    Rt = torch.from_numpy(Rp).cuda()
    for _ in range(500):
        bt.btoep_apply_batched_ptrs(op, "H", [cg.p(0)], [cg.ap(0)], noise_prec, 0.0)
        AP += torch.matmul(P, Rt)  # R symmetric: (R p_t) for every time step t
        bt.btoep_cg_update(cg)
        bt.btoep_cg_poll(cg)
        torch.cuda.synchronize()
        ready, active, iters, rel = bt.btoep_cg_status(cg)
        if ready and active == 0:
            break
    assert ready and active == 0, (iters, rel)
    assert oracle.rel_l2(x[0].cpu().numpy(), x_ref) <= 1e-9
    bt.btoep_cg_end(cg)


@pytest.mark.parametrize("lo_storage", ["f32", "f64"])
def test_stepwise_refined_cg_on_caller_memory(bt, lo_storage):
    """btoep_cg_begin / update / refine / report on caller memory: the FP32 (or FP64) inner
    iteration with FP64 true residuals meets 1e-8 on the oracle's H with the inverse-problem
    scalars (sigma = 1e-2, alpha = 1e-3), the report's residual is the true one, and the
    solution agrees in data space with btoep_cg_solve's."""
    rng = np.random.default_rng(25)
    Nt, Nd, Nm, k = 48, 6, 700, 3
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / (Nt / 7))[:, None, None]
    noise_prec, alpha, rtol = 1e4, 1e-3, 1e-8
    b = noise_prec * oracle.apply_FT(blocks, rng.standard_normal((k, Nt, Nd)))
    hi = make(bt, blocks, "f64")
    lo = make(bt, blocks, lo_storage) if lo_storage != "f64" else hi
    print("case stepwise refined", lo_storage, flush=True)
    x, rep, steps = stepwise_cg(bt, lo, hi, to_dev(b, torch.float64), rtol, noise_prec, alpha, inner_rtol=1e-4,
                                max_iter=2000)
    x = x.cpu().numpy()
    st, res, xs = solve(bt, lo, hi, b, noise_prec, alpha, rtol=rtol, inner_rtol=1e-4)
    assert st == 0
    for r in range(k):
        assert rep[r]["converged"] and rep[r]["rel_residual"] <= rtol and rep[r]["outer_iters"] >= 1, rep
        true = np.linalg.norm(b[r] - oracle.apply_H(blocks, x[r], noise_prec, alpha)) / np.linalg.norm(b[r])
        assert true <= 1.01 * rtol
        assert abs(true - rep[r]["rel_residual"]) <= 0.05 * rtol
        Fd = oracle.apply_F(blocks, x[r] - xs[r])
        assert np.linalg.norm(Fd) <= 1e-6 * np.linalg.norm(oracle.apply_F(blocks, xs[r]))


def test_stepwise_state_arguments_checked(bt):
    blocks = np.ones((8, 2, 3))
    lo = make(bt, blocks, "f32")
    hi = make(bt, blocks, "f64")
    other = make(bt, np.ones((8, 2, 4)), "f64")
    dev, host = bt.btoep_cg_state_size(lo, hi, 2)
    dev_lo, _ = bt.btoep_cg_state_size(lo, None, 2)
    assert dev > dev_lo > 0 and host == 2 * 12 * 8
    with pytest.raises(bt.BtoepError):
        bt.btoep_cg_state_size(lo, other, 2)           # shapes differ
    with pytest.raises(bt.BtoepError):
        bt.btoep_cg_state_size(lo, lo, 2)              # refinement operator must be FP64
    b = torch.zeros((2, 8, 3), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    dm = torch.empty(dev - 256, dtype=torch.uint8, device="cuda")
    hm = torch.empty(host, dtype=torch.uint8, pin_memory=True)
    with pytest.raises(bt.BtoepError, match="workspace"):
        bt.btoep_cg_begin(lo, hi, b, x, 1e-8, 1e-4, dm, hm)
    with pytest.raises(ValueError):
        bt.btoep_cg_begin(lo, hi, b.float(), x.float(), 1e-8, 1e-4, dm, hm)   # refined: FP64 vectors
    assert bt.btoep_cg_workspace_size(lo, hi, 2) > bt.btoep_cg_workspace_size(lo, None, 2)
