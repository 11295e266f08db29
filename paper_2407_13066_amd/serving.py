"""Continuous-batching server for F / F^T / H applies and CG solves on resident operators.

Requests arrive over time, each naming a resident operator, a kind (``F``, ``FT``, ``H`` or
``CG``) and k right-hand sides already in device memory.  The server

* checks each request against its operator (dtype, shape, placement) when it is submitted;
* admits requests first-come-first-served while their device memory (input, output and, for
  CG, the iteration vectors) fits an HBM budget; later arrivals wait until memory frees up;
* forms, every scheduling round, batches per (operator, precision, pipeline, scalars) out of
  whatever is ready: new apply requests and the next H application of every in-flight CG
  solve, up to ``max_batch`` right-hand sides per launch (pointer-array applies, so nothing
  is copied); batches with one-shot applies are launched before batches made only of CG
  iterations;
* launches the batches on several streams, so batches of different operators overlap on the
  device, and enqueues each CG request's vector updates and its scalar poll right behind its
  batch; with graphs on, a batch is one replay of a captured HIP graph for its (operator,
  pipeline, scalars, size, stream), pointed at the batch's vectors through a device address
  table;
* runs CG with FP64 iterative refinement when the executor holds an FP64 copy of the
  operator: inner iterations apply the stored (FP32 / BF16) operator, and whenever the inner
  iteration has stopped, one H application of the FP64 operator to the FP64 iterate gives
  the true residual (section 2.2's system), which decides convergence -- so a CG request's
  reported residual is the true one;
* notices completions without blocking (events, asynchronous CG scalar polls) and records
  arrival-to-completion latency.

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
    rtol: float = 1e-6             # CG only: ||b - H x|| <= rtol ||b|| (true residual when refined)
    max_iter: int = 500            # CG only: inner iterations
    inner_rtol: float = 1e-6       # CG only, refined: inner stop (or below rtol / 2)
    max_outer: int = 10            # CG only, refined: refinement steps
    t_arrival: float = 0.0
    # filled in by the server
    out: object = None
    t_admit: float = None
    t_done: float = None
    iters: int = 0
    outer: int = 0
    converged: bool = None
    rel_residual: list = None      # CG: per right-hand side (true FP64 residual when refined)
    nbytes: int = 0
    _state: object = None          # executor state (CG vectors)
    _ready: object = None          # executor handle the first launch must wait for
    _steps: int = 0                # CG inner steps launched
    _phase: str = "inner"          # CG: "inner" (H_lo p) or "refine" (H_hi x)
    _busy: object = None           # handle of the batch this request is in
    _poll: bool = False            # a CG scalar poll is outstanding
    _poll_due: bool = False        # the next launch ends with a poll
    _finished: bool = False        # CG: no further steps
    _launched: bool = False

    @property
    def k(self):
        return int(self.x.shape[0])

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


class Server:
    def __init__(self, executor, hbm_budget, max_batch=32, n_streams=2, poll_every=1, max_inflight=None,
                 clock=time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.n_streams = int(n_streams)
        # bounded device pipeline: while this many batches are outstanding, new work waits
        # (and accumulates into larger batches) instead of queueing inside the streams
        self.max_inflight = int(max_inflight) if max_inflight else self.n_streams
        # inner CG steps between scalar polls (refinement steps are always followed by one)
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
        self._on_done = None

    # -- arrivals and admission -------------------------------------------------------------
    def submit(self, req):
        if req.kind not in KINDS:
            raise ValueError("unknown request kind %r" % req.kind)
        if req.k > self.max_batch:
            raise ValueError("request %d has %d right-hand sides, more than max_batch" % (req.rid, req.k))
        check = getattr(self.ex, "check", None)
        if check is not None:
            check(req)
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
        if self._on_done is not None:
            self._on_done(req)

    # -- CG progress ------------------------------------------------------------------------
    def _cg_landed(self, req):
        """A poll of `req` has landed: advance its inner / refinement state machine."""
        _, active, iters = self.ex.cg_status(req)
        req.iters = iters
        capped = iters >= req.max_iter or req._steps >= req.max_iter
        refined = self.ex.refined(req)
        if req._phase == "inner":
            if active == 0 or capped:
                if refined:
                    req._phase = "refine"
                else:
                    req._finished = True
                    req.converged = active == 0
            return
        # after a refinement: the true residual decides
        _, res = self.ex.cg_report(req)
        req.rel_residual = [r["rel_residual"] for r in res]
        req.outer = max(r["outer_iters"] for r in res)
        if all(r["converged"] for r in res):
            req._finished, req.converged = True, True
        elif req.outer >= req.max_outer or capped or active == 0:
            req._finished, req.converged = True, False
        else:
            req._phase = "inner"

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
            if req.kind != "CG" or req._busy is not None:
                continue
            if req._poll and self.ex.cg_status(req)[0]:
                req._poll = False
                self._cg_landed(req)
            if req._finished and not req._poll:
                self._release(req, now)

    # -- batching and launch ----------------------------------------------------------------
    def _ready_items(self):
        groups = collections.OrderedDict()
        for req in self.active:
            if req._busy is not None:
                continue
            hi = False
            if req.kind == "CG":
                if req._finished or req._poll:
                    continue
                if req._phase == "inner" and req._steps >= req.max_iter:
                    # cap reached before a poll said so: read the final state
                    continue
                pipe, hi = "H", req._phase == "refine"
            else:
                if req._launched:
                    continue
                pipe = req.kind
            key = (req.op, hi, pipe, req.noise_prec if pipe == "H" else 0.0, req.prior_prec if pipe == "H" else 0.0)
            groups.setdefault(key, []).append(req)
        # groups holding one-shot applies go first (oldest arrival first), then groups made only
        # of CG iterations: a long solve must not hold short requests behind it
        def rank(item):
            reqs = item[1]
            only_cg = all(r.kind == "CG" for r in reqs)
            return (only_cg, min(r.t_arrival for r in reqs))
        return collections.OrderedDict(sorted(groups.items(), key=rank))

    def _launch(self):
        for (op, hi, pipe, noise, prior), reqs in self._ready_items().items():
            batch, nrhs = [], 0
            for req in reqs + [None]:
                if len(self.inflight) >= self.max_inflight:
                    return
                if req is None or nrhs + req.k > self.max_batch:
                    if batch:
                        self._launch_batch(op, hi, pipe, noise, prior, batch, nrhs)
                    batch, nrhs = [], 0
                if req is not None:
                    batch.append(req)
                    nrhs += req.k

    def _launch_batch(self, op, hi, pipe, noise, prior, batch, nrhs):
        stream = self._rr % self.n_streams
        self._rr += 1
        for b in batch:
            if b.kind == "CG":
                if b._phase == "inner":
                    b._steps += 1
                    b._poll_due = (b._steps % self.poll_every == 0 or b._steps >= b.max_iter)
                else:
                    b._poll_due = True
        handle = self.ex.launch(op, pipe, noise, prior, batch, stream, hi=hi)
        self.launches += 1
        self.rhs_applies[pipe + ("64" if hi else "")] += nrhs
        for b in batch:
            b._busy = handle
            b._launched = True
            if b.kind == "CG" and b._poll_due:
                b._poll, b._poll_due = True, False
        self.inflight.append((handle, list(batch)))

    def step(self):
        now = self.clock()
        self._reap(now)
        # CG requests that hit the iteration cap without a landed poll get one of their own
        for req in self.active:
            if (req.kind == "CG" and req._busy is None and not req._poll and not req._finished
                    and req._phase == "inner" and req._steps >= req.max_iter):
                self.ex.cg_poll(req, 0)
                req._poll = True
        self._admit(now)
        self._launch()

    def idle(self):
        return not self.queue and not self.active and not self.inflight

    def run(self, arrivals, t0=None, timeout=None, progress=None, on_done=None):
        """Drive the server through ``arrivals`` (list of (offset seconds, Request)) in real time.
        ``progress(done, total)``, when given, is called every scheduling round; ``on_done(req)``
        as each request completes (a caller that keeps only some answers drops the rest there)."""
        self._on_done = on_done
        arrivals = sorted(arrivals, key=lambda a: a[0])
        t0 = self.clock() if t0 is None else t0
        i = 0
        while i < len(arrivals) or not self.idle():
            now = self.clock()
            if timeout is not None and now - t0 > timeout:
                raise TimeoutError("serving run exceeded %.1f s" % timeout)
            if progress is not None:
                progress(len(self.done), len(arrivals))
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


class _PinnedSlots:
    """Fixed-size slots of pinned host memory for CG scalar polls, allocated in chunks up front
    and recycled, so admitting a CG request does not allocate pinned memory."""

    def __init__(self, torch, slot_bytes, per_chunk=64):
        self.torch, self.slot, self.per_chunk = torch, int(slot_bytes), int(per_chunk)
        self.chunks, self.free = [], []
        self._grow()

    def _grow(self):
        t = self.torch.empty(self.slot * self.per_chunk, dtype=self.torch.uint8, pin_memory=True)
        self.chunks.append(t)
        self.free.extend(t[i * self.slot:(i + 1) * self.slot] for i in range(self.per_chunk))

    def get(self):
        if not self.free:
            self._grow()
        return self.free.pop()

    def put(self, t):
        self.free.append(t)


class GpuExecutor:
    """Runs the server's batches with the HIP library (one workspace per operator and stream).

    ``ops`` maps names to the stored (FP32 / BF16 / FP64) operators the applies use;
    ``ops_hi`` optionally maps the same names to FP64 operators of the same blocks, with which
    CG requests run refined: their right-hand sides and solutions are then FP64 arrays.  With
    ``use_graphs`` every batch is a replay of a graph captured (on first use, or ahead of time
    by ``prepare_graphs``) per (operator, pipeline, scalars, size, stream); otherwise the
    pointer-array apply launches its kernels one by one.  Both run the same kernels.  CG
    states live in device memory from torch's caching allocator and in recycled pinned slots:
    admitting or finishing a request neither allocates through HIP (after warm-up) nor
    waits for the device.
    """

    def __init__(self, ops, n_streams=2, max_batch=32, use_graphs=True, ops_hi=None):
        import torch
        from . import MAX_BATCH, btoep_workspace_size
        self.torch = torch
        self.ops = ops
        self.ops_hi = dict(ops_hi or {})
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.use_graphs = bool(use_graphs)
        self.graphs = {}
        self.ws = {}
        for level, table in (("lo", self.ops), ("hi", self.ops_hi)):
            for name, op in table.items():
                nb = btoep_workspace_size(op, "H", max_batch)
                self.ws[(name, level)] = [torch.empty(nb, dtype=torch.uint8, device="cuda")
                                          for _ in range(n_streams)]
        self.pinned = _PinnedSlots(torch, 8 * 12 * MAX_BATCH)
        self.max_batch = int(max_batch)

    def autotune(self, reps=2, allow_split=False):
        """Pick the kernel variants of every operator, before graphs are captured (a graph
        keeps the kernels it was captured with): the single-vector kernels and transforms of
        all operators, and for the stored FP32 / BF16 operators the matrix-core kernels of each
        right-hand-side bucket up to ``max_batch``.  ``allow_split`` lets FP32 storage take the
        split-BF16 matrix cores: their products stay within the FP32 apply tolerance, but
        their larger error (a few 1e-6 instead of ~1e-6) enters the refinement contraction of
        CG requests squared (eps^2 lambda_max / prior precision), which ill-conditioned
        systems cannot afford, so it is off by default.  Returns the choices."""
        from . import btoep_autotune, btoep_autotune_gemm
        out = {}
        for level, table in (("lo", self.ops), ("hi", self.ops_hi)):
            for name, op in table.items():
                res = {"single": btoep_autotune(op, reps=reps)}
                if op.storage != "f64":
                    res["gemm"] = {k: btoep_autotune_gemm(op, k, allow_split=allow_split, reps=reps)
                                   for k in (8, 16, 32, 64) if k <= self.max_batch}
                out[(name, level)] = res
        return out

    def _op(self, name, hi):
        return self.ops_hi[name] if hi else self.ops[name]

    def _graph(self, op_name, pipe, noise, prior, k, stream_idx, hi=False):
        from . import ApplyGraph
        key = (op_name, hi, pipe, noise, prior, k, stream_idx)
        g = self.graphs.get(key)
        if g is None:
            g = ApplyGraph(self._op(op_name, hi), pipe, k, noise, prior,
                           ws=self.ws[(op_name, "hi" if hi else "lo")][stream_idx])
            self.graphs[key] = g
        return g

    def prepare_graphs(self, pipes, ks, hi=False):
        """Capture ahead of time: ``pipes`` is a list of (operator, pipeline, noise, prior)."""
        for op_name, pipe, noise, prior in pipes:
            for k in ks:
                for si in range(len(self.streams)):
                    self._graph(op_name, pipe, noise, prior, k, si, hi=hi)

    def close(self):
        for g in self.graphs.values():
            g.destroy()
        self.graphs.clear()

    def refined(self, req):
        return req.kind == "CG" and req.op in self.ops_hi

    def input_dtype(self, req):
        return self.torch.float64 if self.refined(req) else self.ops[req.op].vector_dtype

    def check(self, req):
        """Reject a request whose input does not fit its operator before it is admitted."""
        from . import _vec
        if req.op not in self.ops:
            raise ValueError("request %d names unknown operator %r" % (req.rid, req.op))
        op = self.ops[req.op]
        n = op.Nd if req.kind == "FT" else op.Nm
        _vec(op, req.x, (op.Nt, n), "request %d input" % req.rid, dtype=self.input_dtype(req))
        if req.x.dim() != 3:
            raise ValueError("request %d input must be [k][Nt][n]" % req.rid)

    def request_bytes(self, req):
        if req.op not in self.ops:
            raise ValueError("request %d names unknown operator %r" % (req.rid, req.op))
        op = self.ops[req.op]
        vb = 8 if op.storage == "f64" else 4
        n_in = req.k * op.Nt * (op.Nd if req.kind == "FT" else op.Nm)
        n_out = req.k * op.Nt * (op.Nd if req.kind == "F" else op.Nm)
        if req.kind != "CG":
            return (n_in + n_out) * vb
        if self.refined(req):
            return (n_in + n_out) * 8 + self._state_bytes(req)[0]
        return (n_in + n_out) * vb + self._state_bytes(req)[0]

    def _state_bytes(self, req):
        from . import btoep_cg_state_size
        return btoep_cg_state_size(self.ops[req.op], self.ops_hi.get(req.op) if self.refined(req) else None,
                                   req.k)

    def begin(self, req):
        from . import btoep_cg_begin
        torch = self.torch
        op = self.ops[req.op]
        n = op.Nd if req.kind == "F" else op.Nm
        req.out = torch.empty((req.k, op.Nt, n), dtype=self.input_dtype(req) if req.kind == "CG" else op.vector_dtype,
                              device="cuda")
        # the input was written on the caller's stream: the first launch waits for it
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream())
        if req.kind == "CG":
            st = self.streams[0]
            st.wait_event(ready)
            dev_bytes, _ = self._state_bytes(req)
            with torch.cuda.stream(st):
                dev_mem = torch.empty(dev_bytes, dtype=torch.uint8, device="cuda")
            host_mem = self.pinned.get()
            hi = self.ops_hi.get(req.op) if self.refined(req) else None
            req._state = btoep_cg_begin(op, hi, req.x, req.out, req.rtol, req.inner_rtol, dev_mem, host_mem,
                                        stream=st)
            ready = torch.cuda.Event()
            ready.record(st)
        req._ready = ready

    def launch(self, op_name, pipe, noise, prior, batch, stream_idx, hi=False):
        from . import btoep_apply_batched_ptrs, btoep_cg_poll, btoep_cg_refine, btoep_cg_update
        torch = self.torch
        op = self._op(op_name, hi)
        st = self.streams[stream_idx]
        ins, outs = [], []
        for req in batch:
            if req._ready is not None:
                st.wait_event(req._ready)
                req._ready = None
            if req.kind == "CG":
                s = req._state
                if hi:
                    ins += [s.x(r) for r in range(req.k)]
                    outs += [s.hx(r) for r in range(req.k)]
                else:
                    ins += [s.p(r) for r in range(req.k)]
                    outs += [s.ap(r) for r in range(req.k)]
            else:
                rin = req.x.stride(0) * req.x.element_size()
                rout = req.out.stride(0) * req.out.element_size()
                ins += [req.x.data_ptr() + r * rin for r in range(req.k)]
                outs += [req.out.data_ptr() + r * rout for r in range(req.k)]
        if self.use_graphs:
            self._graph(op_name, pipe, noise, prior, len(ins), stream_idx, hi=hi).launch(ins, outs, stream=st)
        else:
            btoep_apply_batched_ptrs(op, pipe, ins, outs, noise, prior,
                                     ws=self.ws[(op_name, "hi" if hi else "lo")][stream_idx], stream=st)
        for req in batch:
            if req.kind == "CG":
                if hi:
                    btoep_cg_refine(req._state, stream=st)
                else:
                    btoep_cg_update(req._state, stream=st)
                if req._poll_due:
                    btoep_cg_poll(req._state, stream=st)
        # The event follows the updates and polls: once it is seen complete, every poll of the
        # batch has landed, and a request is launched again only after that, so consecutive
        # steps of one request need no cross-stream waits.
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

    def cg_report(self, req):
        from . import btoep_cg_report
        return btoep_cg_report(req._state)

    def finish(self, req):
        # the request's work has completed (its last event and poll were seen): its state
        # memory goes back to the caching allocator and the pinned slot to the pool
        if req._state is not None:
            st = req._state
            keep = st.keep
            st.end()
            if keep is not None:
                self.pinned.put(keep[1])
            req._state = None
