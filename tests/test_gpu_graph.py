"""Graph-captured applies and CG iterations through the C-ABI (needs an MI355X).

A graph records the same launches as btoep_apply_batched, so every replay must equal the
launch-by-launch result bit for bit, whatever vectors the device address table names; the
CG solver with graph-replayed inner iterations must return the very same iterate.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import make, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 3e-3}


def vecs(op, which, k, seed):
    n = op.Nd if which == "FT" else op.Nm
    x = synth.vectors(k, op.Nt, n, stream=40 + seed, dtype=np.float64)
    return [to_dev(x[r], op.vector_dtype) for r in range(k)]


def outs_like(op, which, k):
    n = op.Nd if which == "F" else op.Nm
    return [torch.full((op.Nt, n), float("nan"), dtype=op.vector_dtype, device="cuda") for _ in range(k)]


def oracle_apply(blocks, which, x, noise, prior):
    if which == "F":
        return oracle.apply_F(blocks, x)
    if which == "FT":
        return oracle.apply_FT(blocks, x)
    return oracle.apply_H(blocks, x, noise, prior)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("which", ["F", "FT", "H"])
@pytest.mark.parametrize("k", [1, 3, 8])
def test_graph_replays_equal_pointer_batches(bt, storage, which, k):
    Nt, Nd, Nm = 37, 9, 300
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 6, seed=77)
    op = make(bt, blocks, storage)
    noise, prior = 3.0, 0.5
    print("graph case", storage, which, k, flush=True)
    g = bt.ApplyGraph(op, which, k, noise, prior)
    ws = torch.empty(bt.btoep_workspace_size(op, which, k), dtype=torch.uint8, device="cuda")
    prev = None
    for rep in range(3):
        ins = vecs(op, which, k, seed=rep)
        want = outs_like(op, which, k)
        bt.btoep_apply_batched(op, which, ins, want, noise, prior, ws=ws)
        got = outs_like(op, which, k)
        g.launch([t.data_ptr() for t in ins], [t.data_ptr() for t in got])
        torch.cuda.synchronize()
        for r in range(k):
            assert torch.equal(got[r], want[r]), (rep, r)
        # the previous replay's outputs are left alone
        if prev is not None:
            for r in range(k):
                assert torch.equal(prev[0][r], prev[1][r]), ("stale table", rep, r)
        prev = (got, want)
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        del junk
    # a launch without addresses replays on the previous vectors
    for t in got:
        t.fill_(float("nan"))
    g.launch()
    torch.cuda.synchronize()
    for r in range(k):
        assert torch.equal(got[r], want[r]), ("replay on previous vectors", r)
    x = np.stack([t.double().cpu().numpy() for t in ins])
    ref = oracle_apply(blocks, which, x, noise, prior)
    res = np.stack([t.double().cpu().numpy() for t in got])
    assert oracle.rel_l2(res, ref) <= TOL[storage]
    g.destroy()


def test_graph_replayed_back_to_back_on_one_stream(bt):
    """Several replays queued without host waits, each on its own vectors."""
    Nt, Nd, Nm = 64, 12, 1000
    blocks = synth.blocks(Nt, Nd, Nm, tau=10.0, seed=78)
    op = make(bt, blocks, "f32")
    k = 4
    g = bt.ApplyGraph(op, "H", k, 2.0, 1.0)
    ws = torch.empty(bt.btoep_workspace_size(op, "H", k), dtype=torch.uint8, device="cuda")
    runs = []
    for rep in range(5):
        ins = vecs(op, "H", k, seed=10 + rep)
        got = outs_like(op, "H", k)
        g.launch([t.data_ptr() for t in ins], [t.data_ptr() for t in got])
        runs.append((ins, got))
    torch.cuda.synchronize()
    for ins, got in runs:
        want = outs_like(op, "H", k)
        bt.btoep_apply_batched(op, "H", ins, want, 2.0, 1.0, ws=ws)
        torch.cuda.synchronize()
        for r in range(k):
            assert torch.equal(got[r], want[r])


def test_graph_replay_without_vectors_before_any_is_rejected(bt):
    """A graph launched with no vectors before any launch gave some returns INVALID_ARG and
    launches nothing; after one launch with vectors, a vector-less launch replays on them."""
    blocks = synth.blocks(8, 2, 16, tau=4.0, seed=78)
    op = make(bt, blocks, "f32")
    g = bt.ApplyGraph(op, "F", 1)
    with pytest.raises(bt.BtoepError) as e:
        g.launch()
    assert e.value.status == 1
    m = torch.randn((1, 8, 16), device="cuda")
    d = torch.zeros((1, 8, 2), device="cuda")
    g.launch([m.data_ptr()], [d.data_ptr()])
    d.zero_()
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(d, bt.btoep_apply_F(op, m))
    g.destroy()


def test_graph_rejects_small_workspace(bt):
    blocks = synth.blocks(8, 2, 16, tau=4.0, seed=79)
    op = make(bt, blocks, "f32")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(bt.BtoepError) as e:
        bt.ApplyGraph(op, "H", 2, ws=ws)
    assert e.value.status == 6


@pytest.mark.parametrize("lo_storage", ["f64", "f32"])
def test_cg_graph_iterations_equal_launch_by_launch(bt, lo_storage):
    rng = np.random.default_rng(31)
    Nt, Nd, Nm, k = 40, 5, 600, 2
    blocks = rng.standard_normal((Nt, Nd, Nm)) * np.exp(-np.arange(Nt) / 6.0)[:, None, None]
    b = to_dev(rng.standard_normal((k, Nt, Nm)), torch.float64)
    lo = make(bt, blocks, lo_storage)
    hi = make(bt, blocks, "f64") if lo_storage != "f64" else None
    out = {}
    for use_graph in (False, True):
        x = torch.zeros_like(b)
        st, res = bt.btoep_cg_solve(lo, hi, b, x, 4.0, 0.1, rtol=1e-9, inner_rtol=1e-5, max_inner=400,
                                    check_every=3, use_graph=use_graph)
        torch.cuda.synchronize()
        out[use_graph] = (st, res, x.cpu())
    assert out[True][0] == out[False][0] == 0
    assert out[True][1] == out[False][1]
    assert torch.equal(out[True][2], out[False][2])
