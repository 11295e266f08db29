"""Adapters that run the HIP path on numpy inputs (used by the GPU tests)."""
import numpy as np
import torch


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def make(bt, blocks, storage):
    return bt.btoep_create(np.ascontiguousarray(blocks, dtype=np.float64), storage)


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
