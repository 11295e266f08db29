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
    """Executes each batch with the oracle; a batch 'completes' `delay` seconds after launch.

    CG follows the library's stepwise protocol.  With ``refine`` the inner iterations apply H
    built from the blocks rounded to float32 (a stand-in for the stored low-precision operator)
    and every refinement step forms the true residual with the exact FP64 operator, so that
    refinement has something to correct."""

    def __init__(self, ops, clock, delay=5e-3, vbytes=4, refine=False):
        self.ops, self.clock, self.delay, self.vb, self.refine = ops, clock, delay, vbytes, refine
        self.ops_lo = {n: b.astype(np.float32).astype(np.float64) for n, b in ops.items()}
        self.batches = []

    def refined(self, req):
        return self.refine and req.kind == "CG"

    def request_bytes(self, req):
        Nt, Nd, Nm = self.ops[req.op].shape
        n_in = req.k * Nt * (Nd if req.kind == "FT" else Nm)
        n_out = req.k * Nt * (Nd if req.kind == "F" else Nm)
        return (n_in + n_out + (3 * req.k * Nt * Nm if req.kind == "CG" else 0)) * self.vb

    @staticmethod
    def _dot(a, b):
        return (a * b).sum(axis=(1, 2))

    def _restart(self, req, res, outer_test):
        st = req._state
        st["r"] = res.copy()
        st["p"] = res.copy()
        st["rr"] = self._dot(res, res)
        floor = 0.25 * req.rtol ** 2 * st["bb"] if self.refined(req) else 0.0
        inner2 = req.inner_rtol ** 2 if self.refined(req) else req.rtol ** 2
        st["th"] = np.maximum(inner2 * st["rr"], floor)
        st["act"] = (st["rh"] > outer_test * st["bb"]) & (st["rr"] > st["th"])

    def begin(self, req):
        if req.kind == "CG":
            b = np.asarray(req.x, dtype=np.float64)
            bb = self._dot(b, b)
            req._state = {"b": b, "x": np.zeros_like(b), "bb": bb, "rh": bb.copy(), "it": np.zeros(req.k, int),
                          "outer": 0, "snap": None}
            self._restart(req, b, req.rtol ** 2 if self.refined(req) else 0.0)

    def launch(self, op, pipe, noise, prior, batch, stream, hi=False):
        blocks = self.ops[op]
        self.batches.append((op, pipe + ("64" if hi else ""), sum(r.k for r in batch), [r.rid for r in batch]))
        for req in batch:
            if req.kind == "CG":
                st = req._state
                if hi:
                    res = st["b"] - oracle.apply_H(blocks, st["x"], noise, prior)
                    st["rh"] = self._dot(res, res)
                    st["outer"] += 1
                    self._restart(req, res, req.rtol ** 2)
                else:
                    lo = self.ops_lo[op] if self.refined(req) else blocks
                    act = st["act"]
                    Ap = oracle.apply_H(lo, st["p"], noise, prior)
                    al = np.where(act, st["rr"] / self._dot(st["p"], Ap), 0.0)
                    st["x"] += al[:, None, None] * st["p"]
                    st["r"] -= al[:, None, None] * Ap
                    rrn = self._dot(st["r"], st["r"])
                    be = np.where(act, rrn / st["rr"], 0.0)
                    st["p"] = np.where(act[:, None, None], st["r"] + be[:, None, None] * st["p"], st["p"])
                    st["it"] += act
                    st["rr"] = np.where(act, rrn, st["rr"])
                    st["act"] = act & (rrn > st["th"])
                if req._poll_due:
                    self.cg_poll(req, stream)
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
        res2 = st["rh"] if self.refined(req) else st["rr"]
        results = [dict(inner_iters=int(st["it"][r]), outer_iters=st["outer"], matvecs=0,
                        converged=bool(res2[r] <= req.rtol ** 2 * st["bb"][r]),
                        rel_residual=float(np.sqrt(res2[r] / st["bb"][r]))) for r in range(req.k)]
        st["snap"] = (self.clock.t + self.delay, int(st["act"].sum()), int(st["it"].max()), results)

    def cg_status(self, req):
        t, active, iters, _ = req._state["snap"]
        return (self.clock.t >= t), active, iters

    def cg_report(self, req):
        t, _, _, results = req._state["snap"]
        return (self.clock.t >= t), results

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


def test_refined_cg_meets_the_true_residual():
    """With a float32-rounded inner operator, CG converges only through refinement: every
    solve ends with a true (exact-operator) residual at or below rtol, after at least one
    refinement step, and the refinement applies show up as their own pipeline."""
    rng = np.random.default_rng(5)
    ops = make_ops(rng)
    clock = FakeClock()
    ex = OracleExecutor(ops, clock, refine=True)
    srv = Server(ex, hbm_budget=1 << 30, max_batch=8, n_streams=2, clock=clock)
    arrivals = make_requests(rng, ops, 12, kinds=("CG", "H"))
    for _, req in arrivals:
        req.rtol, req.inner_rtol = 1e-12, 1e-3
    srv.run(arrivals, t0=0.0)
    assert srv.idle() and srv.used == 0
    for _, req in arrivals:
        if req.kind != "CG":
            continue
        assert req.converged and req.outer >= 1
        for r in range(req.k):
            res = req.x[r] - oracle.apply_H(ops[req.op], req.out[r], 2.0, 1.0)
            assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(req.x[r]) * (1 + 1e-9)
            assert req.rel_residual[r] <= 1e-12
    assert srv.rhs_applies["H64"] > 0 and any(p == "H64" for (_, p, _, _) in ex.batches)


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
