"""The continuous-batching scheduler driven by a CPU executor built on the FP64 oracle.

Checks admission by HBM budget, batching across requests, CG stepping and completion,
latency bookkeeping and error paths without a GPU (a fake clock makes it deterministic).
"""
import numpy as np
import pytest

import oracle
from paper_2407_13066_amd.serving import Request, Server, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3   # every scheduling round advances 1 ms
        return self.t


class OracleExecutor:
    """Executes each batch with the oracle; a batch 'completes' `delay` seconds after launch."""

    def __init__(self, ops, clock, delay=5e-3, vbytes=4):
        self.ops, self.clock, self.delay, self.vb = ops, clock, delay, vbytes
        self.batches = []

    def request_bytes(self, req):
        Nt, Nd, Nm = self.ops[req.op].shape
        n_in = req.k * Nt * (Nd if req.kind == "FT" else Nm)
        n_out = req.k * Nt * (Nd if req.kind == "F" else Nm)
        return (n_in + n_out + (3 * req.k * Nt * Nm if req.kind == "CG" else 0)) * self.vb

    def begin(self, req):
        if req.kind == "CG":
            b = np.asarray(req.x, dtype=np.float64)
            req._state = {"x": np.zeros_like(b), "r": b.copy(), "p": b.copy(), "rr": (b * b).sum(axis=(1, 2)),
                          "bb": (b * b).sum(axis=(1, 2)), "it": np.zeros(req.k, int), "snap": None}

    def launch(self, op, pipe, noise, prior, batch, stream):
        blocks = self.ops[op]
        self.batches.append((op, pipe, sum(r.k for r in batch), [r.rid for r in batch]))
        for req in batch:
            if req.kind == "CG":
                st = req._state
                act = st["rr"] > req.rtol ** 2 * st["bb"]
                Ap = oracle.apply_H(blocks, st["p"], noise, prior)
                pAp = (st["p"] * Ap).sum(axis=(1, 2))
                al = np.where(act, st["rr"] / pAp, 0.0)
                st["x"] += al[:, None, None] * st["p"]
                st["r"] -= al[:, None, None] * Ap
                rrn = (st["r"] * st["r"]).sum(axis=(1, 2))
                be = np.where(act, rrn / st["rr"], 0.0)
                st["p"] = np.where(act[:, None, None], st["r"] + be[:, None, None] * st["p"], st["p"])
                st["it"] += act
                st["rr"] = np.where(act, rrn, st["rr"])
            elif pipe == "F":
                req.out = oracle.apply_F(blocks, req.x)
            elif pipe == "FT":
                req.out = oracle.apply_FT(blocks, req.x)
            else:
                req.out = oracle.apply_H(blocks, req.x, noise, prior)
        return self.clock.t + self.delay

    def is_done(self, handle):
        return self.clock.t >= handle

    def cg_poll(self, req, stream):
        st = req._state
        st["snap"] = (self.clock.t + self.delay, int((st["rr"] > req.rtol ** 2 * st["bb"]).sum()), int(st["it"].max()))

    def cg_status(self, req):
        t, active, iters = req._state["snap"]
        return (self.clock.t >= t), active, iters

    def finish(self, req):
        if req.kind == "CG":
            req.out = req._state["x"]
            req._state = None


def make_ops(rng):
    return {"A": rng.standard_normal((6, 2, 9)), "B": rng.standard_normal((5, 3, 7))}


def make_requests(rng, ops, n, kinds=("F", "FT", "H", "CG")):
    arrivals = []
    for i in range(n):
        name = ["A", "B"][i % 2]
        Nt, Nd, Nm = ops[name].shape
        kind = kinds[i % len(kinds)]
        k = int(rng.integers(1, 4))
        x = rng.standard_normal((k, Nt, Nd if kind == "FT" else Nm))
        req = Request(rid=i, op=name, kind=kind, x=x, noise_prec=2.0, prior_prec=1.0, rtol=1e-10, max_iter=200)
        arrivals.append((0.002 * i, req))
    return arrivals


def test_results_match_solo_oracle_and_everything_completes():
    rng = np.random.default_rng(0)
    ops = make_ops(rng)
    clock = FakeClock()
    ex = OracleExecutor(ops, clock)
    srv = Server(ex, hbm_budget=1 << 30, max_batch=8, n_streams=2, poll_every=3, clock=clock)
    arrivals = make_requests(rng, ops, 24)
    done = srv.run(arrivals, t0=0.0)
    assert len(done) == 24 and srv.idle() and srv.used == 0
    for _, req in arrivals:
        blocks = ops[req.op]
        if req.kind == "F":
            want = oracle.apply_F(blocks, req.x)
        elif req.kind == "FT":
            want = oracle.apply_FT(blocks, req.x)
        elif req.kind == "H":
            want = oracle.apply_H(blocks, req.x, 2.0, 1.0)
        else:
            assert req.converged and req.iters > 0
            want = np.stack([np.linalg.solve(
                2.0 * (A := __import__("tests.pins", fromlist=["dense_matrix"]).dense_matrix(blocks)).T @ A
                + np.eye(A.shape[1]), b.ravel()).reshape(b.shape) for b in req.x])
            assert oracle.rel_l2(req.out, want) < 1e-8
            continue
        assert oracle.rel_l2(req.out, want) == 0.0
        assert req.latency is not None and req.latency > 0


def test_requests_are_batched_across_arrivals():
    rng = np.random.default_rng(1)
    ops = make_ops(rng)
    clock = FakeClock()
    ex = OracleExecutor(ops, clock, delay=0.02)
    srv = Server(ex, hbm_budget=1 << 30, max_batch=16, n_streams=1, clock=clock)
    arrivals = make_requests(rng, ops, 20, kinds=("H",))
    srv.run(arrivals, t0=0.0)
    assert srv.launches < 20
    assert any(len(rids) > 1 for (_, _, _, rids) in ex.batches)
    assert all(nrhs <= 16 for (_, _, nrhs, _) in ex.batches)
    assert srv.rhs_applies["H"] == sum(r.k for _, r in arrivals)


def test_admission_respects_the_memory_budget():
    rng = np.random.default_rng(2)
    ops = make_ops(rng)
    clock = FakeClock()
    ex = OracleExecutor(ops, clock, delay=0.03)
    arrivals = make_requests(rng, ops, 16, kinds=("H", "CG"))
    biggest = max(ex.request_bytes(r) for _, r in arrivals)
    budget = 2 * biggest
    srv = Server(ex, hbm_budget=budget, max_batch=8, clock=clock)
    srv.run(arrivals, t0=0.0)
    assert srv.peak_used <= budget
    assert any(r.t_admit > r.t_arrival for _, r in arrivals)   # someone had to wait for memory
    lat = [r.latency for _, r in arrivals]
    assert percentile(lat, 50) <= percentile(lat, 99) <= max(lat)


def test_cg_stops_at_max_iter_without_converging():
    rng = np.random.default_rng(3)
    ops = make_ops(rng)
    clock = FakeClock()
    ex = OracleExecutor(ops, clock)
    srv = Server(ex, hbm_budget=1 << 30, poll_every=4, clock=clock)
    b = rng.standard_normal((1, 6, 9))
    req = Request(rid=0, op="A", kind="CG", x=b, noise_prec=1e4, prior_prec=1e-6, rtol=1e-30, max_iter=6)
    srv.run([(0.0, req)], t0=0.0, timeout=100.0)
    assert req.converged is False and req.iters == 6


def test_submission_errors():
    rng = np.random.default_rng(4)
    ops = make_ops(rng)
    clock = FakeClock()
    ex = OracleExecutor(ops, clock)
    srv = Server(ex, hbm_budget=100, max_batch=2, clock=clock)
    with pytest.raises(ValueError):
        srv.submit(Request(rid=0, op="A", kind="X", x=np.zeros((1, 6, 9))))
    with pytest.raises(ValueError):
        srv.submit(Request(rid=1, op="A", kind="H", x=np.zeros((3, 6, 9))))   # more than max_batch
    with pytest.raises(ValueError):
        srv.submit(Request(rid=2, op="A", kind="H", x=np.zeros((1, 6, 9))))   # over the budget


def test_percentile_nearest_rank():
    assert percentile([5, 1, 3, 2, 4], 50) == 3
    assert percentile(list(range(1, 101)), 99) == 99
    assert percentile([], 50) is None
