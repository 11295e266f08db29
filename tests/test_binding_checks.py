"""Host-side argument checks of the Python binding and the server (no GPU, no library call):
a tensor of the wrong dtype, shape, layout or placement is rejected before any pointer
reaches the C interface, where it could be read or written out of bounds on the device."""
import pytest
import torch

import paper_2407_13066_amd as bt
from paper_2407_13066_amd.serving import GpuExecutor, Request, Server


def fake_op(storage="f32", Nt=8, Nd=3, Nm=5):
    info = dict(Nt=Nt, Nd=Nd, Nm=Nm, L=2 * Nt, nfreq=Nt + 1, ldF=8, storage=storage,
                vector="f64" if storage == "f64" else "f32", fhat_bytes=0, device=0)
    return bt.Op(None, info)


def test_vector_checks():
    op = fake_op()
    good = torch.zeros((2, 8, 5), dtype=torch.float32)
    with pytest.raises(ValueError, match="dtype"):
        bt._vec(op, good.double(), (8, 5), "m")
    with pytest.raises(ValueError, match="shape"):
        bt._vec(op, torch.zeros((2, 8, 4)), (8, 5), "m")
    with pytest.raises(ValueError, match="shape"):
        bt._vec(op, torch.zeros((2, 8, 5)), (8, 5), "m", single=True)
    with pytest.raises(ValueError, match="contiguous"):
        bt._vec(op, torch.zeros((2, 5, 8)).transpose(1, 2), (8, 5), "m")
    with pytest.raises(ValueError, match="CUDA"):
        bt._vec(op, good, (8, 5), "m")
    with pytest.raises(TypeError):
        bt._vec(op, [0.0] * 40, (8, 5), "m")


def test_apply_and_cg_reject_bad_tensors():
    op = fake_op()
    with pytest.raises(ValueError, match="shape"):
        bt.btoep_apply_F(op, torch.zeros((1, 8, 6)))
    with pytest.raises(ValueError, match="dtype"):
        bt.btoep_apply_H(op, torch.zeros((1, 8, 5), dtype=torch.float64))
    with pytest.raises(ValueError, match="shape"):
        bt.btoep_apply_batched(op, "FT", [torch.zeros((8, 5))], [torch.zeros((8, 5))])
    with pytest.raises(ValueError):
        bt.btoep_apply_batched(op, "X", [torch.zeros((8, 5))], [torch.zeros((8, 3))])
    b = torch.zeros((2, 8, 5), dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        bt.btoep_cg_solve(op, None, b.float(), b.float(), 1.0, 1.0)
    with pytest.raises(ValueError, match="shape"):
        bt.btoep_cg_solve(op, None, b, torch.zeros((2, 8, 6), dtype=torch.float64), 1.0, 1.0)


def test_server_rejects_requests_that_do_not_fit_their_operator():
    ex = GpuExecutor.__new__(GpuExecutor)       # no streams or workspaces: only the checks
    ex.ops = {"A": fake_op()}
    srv = Server(ex, hbm_budget=1 << 30)
    with pytest.raises(ValueError, match="unknown operator"):
        srv.submit(Request(rid=0, op="Z", kind="F", x=torch.zeros((1, 8, 5))))
    with pytest.raises(ValueError, match="dtype"):
        srv.submit(Request(rid=1, op="A", kind="H", x=torch.zeros((1, 8, 5), dtype=torch.float64)))
    with pytest.raises(ValueError, match="shape"):
        srv.submit(Request(rid=2, op="A", kind="FT", x=torch.zeros((1, 8, 5))))   # F^T takes [k][Nt][Nd]
    with pytest.raises(ValueError, match="CUDA"):
        srv.submit(Request(rid=3, op="A", kind="F", x=torch.zeros((1, 8, 5))))
    assert not srv.queue
