"""Continuous-batching server for F / F^T / H applies and CG solves on resident operators.

Requests arrive over time, each naming a resident operator, a kind (``F``, ``FT``, ``H`` or
``CG``) and k right-hand sides already in device memory.  The server

* admits requests first-come-first-served while their device memory (input, output and, for
  CG, the iteration vectors) fits an HBM budget; later arrivals wait until memory frees up;
* forms, every scheduling round, batches per (operator, pipeline, scalars) out of whatever is
  ready: new apply requests and the next H application of every in-flight CG solve, up to
  ``max_batch`` right-hand sides per launch (pointer-array applies, so nothing is copied);
  batches with one-shot applies are launched before batches made only of CG iterations;
* launches the batches on several streams, so batches of different operators overlap on the
  device, and enqueues each CG request's vector updates right behind its batch; with graphs
  on, a batch is one replay of a captured HIP graph for its (operator, pipeline, scalars,
  size, stream), pointed at the batch's vectors through a device address table;
* notices completions without blocking (events, asynchronous CG residual polls) and
  records arrival-to-completion latency.

Every right-hand side is computed independently by the kernels, so a request's result does
not depend on what it was batched with beyond the rounding differences between the
single-vector and matrix-core kernels.

The device work goes through an *executor* (``GpuExecutor`` drives the HIP library); the
scheduler itself only does bookkeeping, which lets it be exercised with any executor.
"""
import collections
import dataclasses
import time

KINDS = ("F", "FT", "H", "CG")


@dataclasses.dataclass
class Request:
    rid: int
    op: str
    kind: str
    x: object                      # input [k][Nt][n] on the device (m, or d for FT; b for CG)
    noise_prec: float = 1.0
    prior_prec: float = 1.0
    rtol: float = 1e-6             # CG only (recurrence residual)
    max_iter: int = 500            # CG only
    t_arrival: float = 0.0
    # filled in by the server
    out: object = None
    t_admit: float = None
    t_done: float = None
    iters: int = 0
    converged: bool = None
    nbytes: int = 0
    _state: object = None          # executor state (CG vectors)
    _ready: object = None          # executor handle the first launch must wait for
    _steps: int = 0                # CG steps launched
    _busy: object = None           # handle of the batch this request is in
    _poll: bool = False            # a CG residual poll is outstanding
    _finished: bool = False        # CG: no further steps
    _launched: bool = False

    @property
    def k(self):
        return int(self.x.shape[0])

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


class Server:
    def __init__(self, executor, hbm_budget, max_batch=32, n_streams=2, poll_every=4, max_inflight=None,
                 clock=time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.n_streams = int(n_streams)
        # bounded device pipeline: while this many batches are outstanding, new work waits
        # (and accumulates into larger batches) instead of queueing inside the streams
        self.max_inflight = int(max_inflight) if max_inflight else self.n_streams
        self.poll_every = int(poll_every)
        self.clock = clock
        self.queue = collections.deque()
        self.active = []
        self.done = []
        self.inflight = []           # (handle, [requests])
        self.used = 0
        self.peak_used = 0
        self._rr = 0
        self.rhs_applies = collections.Counter()   # right-hand-side applications per pipeline
        self.launches = 0

    # -- arrivals and admission -------------------------------------------------------------
    def submit(self, req):
        if req.kind not in KINDS:
            raise ValueError("unknown request kind %r" % req.kind)
        if req.k > self.max_batch:
            raise ValueError("request %d has %d right-hand sides, more than max_batch" % (req.rid, req.k))
        req.nbytes = self.ex.request_bytes(req)
        if req.nbytes > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget" % (req.rid, req.nbytes))
        self.queue.append(req)

    def _admit(self, now):
        while self.queue and self.used + self.queue[0].nbytes <= self.budget:
            req = self.queue.popleft()
            self.used += req.nbytes
            self.peak_used = max(self.peak_used, self.used)
            req.t_admit = now
            self.ex.begin(req)
            self.active.append(req)

    def _release(self, req, now):
        req.t_done = now
        self.ex.finish(req)
        self.used -= req.nbytes
        self.active.remove(req)
        self.done.append(req)

    # -- completions ------------------------------------------------------------------------
    def _reap(self, now):
        still = []
        for handle, reqs in self.inflight:
            if not self.ex.is_done(handle):
                still.append((handle, reqs))
                continue
            for req in reqs:
                req._busy = None
                if req.kind != "CG":
                    self._release(req, now)
        self.inflight = still
        for req in list(self.active):
            if req.kind != "CG":
                continue
            if req._poll:
                ready, active, iters = self.ex.cg_status(req)
                if ready:
                    req._poll = False
                    req.iters = iters
                    if active == 0 or iters >= req.max_iter:
                        req._finished = True
                        req.converged = active == 0
            if (not req._finished and not req._poll and req._busy is None and req._steps >= req.max_iter):
                self.ex.cg_poll(req, 0)  # its last step is complete: read the final state
                req._poll = True
            if req._finished and req._busy is None and not req._poll:
                self._release(req, now)

    # -- batching and launch ----------------------------------------------------------------
    def _ready_items(self):
        groups = collections.OrderedDict()
        for req in self.active:
            if req._busy is not None:
                continue
            if req.kind == "CG":
                if req._finished or req._steps >= req.max_iter:
                    continue
                pipe = "H"
            else:
                if req._launched:
                    continue
                pipe = req.kind
            key = (req.op, pipe, req.noise_prec if pipe == "H" else 0.0, req.prior_prec if pipe == "H" else 0.0)
            groups.setdefault(key, []).append(req)
        # groups holding one-shot applies go first (oldest arrival first), then groups made only
        # of CG iterations: a long solve must not hold short requests behind it
        def rank(item):
            reqs = item[1]
            only_cg = all(r.kind == "CG" for r in reqs)
            return (only_cg, min(r.t_arrival for r in reqs))
        return collections.OrderedDict(sorted(groups.items(), key=rank))

    def _launch(self):
        for (op, pipe, noise, prior), reqs in self._ready_items().items():
            batch, nrhs = [], 0
            for req in reqs + [None]:
                if len(self.inflight) >= self.max_inflight:
                    return
                if req is None or nrhs + req.k > self.max_batch:
                    if batch:
                        stream = self._rr % self.n_streams
                        self._rr += 1
                        handle = self.ex.launch(op, pipe, noise, prior, batch, stream)
                        self.launches += 1
                        self.rhs_applies[pipe] += nrhs
                        for b in batch:
                            b._busy = handle
                            b._launched = True
                            if b.kind == "CG":
                                b._steps += 1
                                due = b._steps % self.poll_every == 0 or b._steps >= b.max_iter
                                if due and not b._poll:
                                    self.ex.cg_poll(b, stream)
                                    b._poll = True
                        self.inflight.append((handle, list(batch)))
                    batch, nrhs = [], 0
                if req is not None:
                    batch.append(req)
                    nrhs += req.k

    def step(self):
        now = self.clock()
        self._reap(now)
        self._admit(now)
        self._launch()

    def idle(self):
        return not self.queue and not self.active and not self.inflight

    def run(self, arrivals, t0=None, timeout=None):
        """Drive the server through ``arrivals`` (list of (offset seconds, Request)) in real time."""
        arrivals = sorted(arrivals, key=lambda a: a[0])
        t0 = self.clock() if t0 is None else t0
        i = 0
        while i < len(arrivals) or not self.idle():
            now = self.clock()
            if timeout is not None and now - t0 > timeout:
                raise TimeoutError("serving run exceeded %.1f s" % timeout)
            while i < len(arrivals) and t0 + arrivals[i][0] <= now:
                req = arrivals[i][1]
                req.t_arrival = t0 + arrivals[i][0]
                self.submit(req)
                i += 1
            self.step()
        return self.done


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return None
    idx = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[idx]


class GpuExecutor:
    """Runs the server's batches with the HIP library (one workspace per operator and stream).

    With ``use_graphs`` every batch is a replay of a graph captured (on first use, or ahead of
    time by ``prepare_graphs``) per (operator, pipeline, scalars, size, stream); otherwise the
    pointer-array apply launches its kernels one by one.  Both run the same kernels.
    """

    def __init__(self, ops, n_streams=2, max_batch=32, use_graphs=True):
        import torch
        from . import btoep_workspace_size
        self.torch = torch
        self.ops = ops
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.use_graphs = bool(use_graphs)
        self.graphs = {}
        self.ws = {}
        for name, op in ops.items():
            nb = btoep_workspace_size(op, "H", max_batch)
            self.ws[name] = [torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(n_streams)]

    def _graph(self, op_name, pipe, noise, prior, k, stream_idx):
        from . import ApplyGraph
        key = (op_name, pipe, noise, prior, k, stream_idx)
        g = self.graphs.get(key)
        if g is None:
            g = ApplyGraph(self.ops[op_name], pipe, k, noise, prior, ws=self.ws[op_name][stream_idx])
            self.graphs[key] = g
        return g

    def prepare_graphs(self, pipes, ks):
        """Capture ahead of time: ``pipes`` is a list of (operator, pipeline, noise, prior)."""
        for op_name, pipe, noise, prior in pipes:
            for k in ks:
                for si in range(len(self.streams)):
                    self._graph(op_name, pipe, noise, prior, k, si)

    def close(self):
        for g in self.graphs.values():
            g.destroy()
        self.graphs.clear()

    def request_bytes(self, req):
        op = self.ops[req.op]
        vb = 8 if op.storage == "f64" else 4
        n_in = req.k * op.Nt * (op.Nd if req.kind == "FT" else op.Nm)
        n_out = req.k * op.Nt * (op.Nd if req.kind == "F" else op.Nm)
        extra = 3 * req.k * op.Nt * op.Nm if req.kind == "CG" else 0
        return (n_in + n_out + extra) * vb

    def begin(self, req):
        from . import btoep_cg_start
        torch = self.torch
        op = self.ops[req.op]
        n = op.Nd if req.kind == "F" else op.Nm
        req.out = torch.empty((req.k, op.Nt, n), dtype=op.vector_dtype, device="cuda")
        # the input was written on the caller's stream: the first launch waits for it
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream())
        if req.kind == "CG":
            st = self.streams[0]
            st.wait_event(ready)
            req._state = btoep_cg_start(op, req.x, req.out, req.rtol, req.noise_prec, req.prior_prec, stream=st)
            ready = torch.cuda.Event()
            ready.record(st)
        req._ready = ready

    def launch(self, op_name, pipe, noise, prior, batch, stream_idx):
        from . import btoep_apply_batched_ptrs, btoep_cg_update
        torch = self.torch
        op = self.ops[op_name]
        st = self.streams[stream_idx]
        ins, outs = [], []
        for req in batch:
            if req._ready is not None:
                st.wait_event(req._ready)
                req._ready = None
            if req.kind == "CG":
                ins += [req._state.p(r) for r in range(req.k)]
                outs += [req._state.ap(r) for r in range(req.k)]
            else:
                rin = req.x.stride(0) * req.x.element_size()
                rout = req.out.stride(0) * req.out.element_size()
                ins += [req.x.data_ptr() + r * rin for r in range(req.k)]
                outs += [req.out.data_ptr() + r * rout for r in range(req.k)]
        if self.use_graphs:
            self._graph(op_name, pipe, noise, prior, len(ins), stream_idx).launch(ins, outs, stream=st)
        else:
            btoep_apply_batched_ptrs(op, pipe, ins, outs, noise, prior, ws=self.ws[op_name][stream_idx], stream=st)
        for req in batch:
            if req.kind == "CG":
                btoep_cg_update(req._state, stream=st)
        # A request is launched again only after this event has been seen complete, so
        # consecutive steps of one request need no cross-stream waits.
        ev = torch.cuda.Event()
        ev.record(st)
        return ev

    def is_done(self, handle):
        return handle.query()

    def cg_poll(self, req, stream_idx):
        from . import btoep_cg_poll
        btoep_cg_poll(req._state, stream=self.streams[stream_idx])

    def cg_status(self, req):
        from . import btoep_cg_status
        ready, active, iters, _ = btoep_cg_status(req._state)
        return ready, active, iters

    def finish(self, req):
        if req._state is not None:
            req._state.end()
            req._state = None
