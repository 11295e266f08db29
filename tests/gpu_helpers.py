"""Adapters that run the HIP path on numpy inputs (used by the GPU tests)."""
import numpy as np
import torch


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def make(bt, blocks, storage):
    """Operator of `storage`; "f32split" is FP32 storage whose several-right-hand-side products
    run on the BF16 matrix cores with the three-term split."""
    op = bt.btoep_create(np.ascontiguousarray(blocks, dtype=np.float64), "f32" if storage == "f32split" else storage)
    if storage == "f32split":
        bt.btoep_set_gemm(op, True)
    return op


def gpu_F(bt, storage):
    def F(blocks, m):
        op = make(bt, blocks, storage)
        out = bt.btoep_apply_F(op, to_dev(m, op.vector_dtype))
        torch.cuda.synchronize()
        return out.double().cpu().numpy()
    return F


def gpu_FT(bt, storage):
    def FT(blocks, d):
        op = make(bt, blocks, storage)
        out = bt.btoep_apply_FT(op, to_dev(d, op.vector_dtype))
        torch.cuda.synchronize()
        return out.double().cpu().numpy()
    return FT


def gpu_H(bt, storage):
    def H(blocks, m, noise_prec=1.0, prior_prec=1.0):
        op = make(bt, blocks, storage)
        out = bt.btoep_apply_H(op, to_dev(m, op.vector_dtype), noise_prec, prior_prec)
        torch.cuda.synchronize()
        return out.double().cpu().numpy()
    return H


def stepwise_cg(bt, op, op_hi, b, rtol, noise_prec, prior_prec, inner_rtol=1e-6, max_iter=500, max_outer=10):
    """Runs one stepwise CG solve alone through the C-ABI (caller memory, btoep_cg_begin):
    the caller applies H_lo to p after each poll that shows inner work left and, with an
    FP64 refinement operator, H_hi to x whenever the inner iteration has stopped.
    Returns (x, per-right-hand-side report, inner H applications)."""
    k = b.shape[0]
    dev, host = bt.btoep_cg_state_size(op, op_hi, k)
    dm = torch.empty(dev, dtype=torch.uint8, device="cuda")
    hm = torch.empty(host, dtype=torch.uint8, pin_memory=True)
    x = torch.empty_like(b)
    cg = bt.btoep_cg_begin(op, op_hi, b, x, rtol, inner_rtol, dm, hm)
    steps, report = 0, None
    while True:
        while steps < max_iter:
            bt.btoep_apply_batched_ptrs(op, "H", [cg.p(r) for r in range(k)], [cg.ap(r) for r in range(k)],
                                        noise_prec, prior_prec)
            bt.btoep_cg_update(cg)
            bt.btoep_cg_poll(cg)
            torch.cuda.synchronize()
            steps += 1
            ready, active, _, _ = bt.btoep_cg_status(cg)
            assert ready
            if active == 0:
                break
        if op_hi is None:
            torch.cuda.synchronize()
            break
        bt.btoep_apply_batched_ptrs(op_hi, "H", [cg.x(r) for r in range(k)], [cg.hx(r) for r in range(k)],
                                    noise_prec, prior_prec)
        bt.btoep_cg_refine(cg)
        bt.btoep_cg_poll(cg)
        torch.cuda.synchronize()
        ready, report = bt.btoep_cg_report(cg)
        assert ready
        if all(r["converged"] for r in report) or report[0]["outer_iters"] >= max_outer or steps >= max_iter:
            break
    if report is None:
        bt.btoep_cg_poll(cg)
        torch.cuda.synchronize()
        _, report = bt.btoep_cg_report(cg)
    cg.end()
    return x, report, steps


def power_sigma2(apply_F, apply_FT, shape, iters=60, seed=0):
    """Largest eigenvalue of F^T F by power iteration (the oracle's F and F^T)."""
    v = np.random.default_rng(seed).standard_normal(shape)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = apply_FT(apply_F(v))
        lam = float(np.vdot(v, w))
        v = w / np.linalg.norm(w)
    return lam
