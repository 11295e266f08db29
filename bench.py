#!/usr/bin/env python3
"""Benchmark of the Hessian action H m = F^T(noise_prec F m) + prior_prec m on one MI355X.

Workload: FP32-complex stored operator, Nt=420 time blocks of Nd=100 x Nm=65536
(F_k = N(0,1) exp(-k/60), seeded), one right-hand side m ~ N(0,1), noise_prec =
prior_prec = 1.  One step = one H application (both passes over the 22 GB operator plus
the transforms), inputs already resident in device memory.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak


def log(*a):
    print("[bench %6.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


T0 = time.time()


def algorithmic_bytes(Nt, Nd, Nm, nfreq, nspan, sb, vb):
    """Bytes each kernel of one H application must move (see the design notes):
    sb = bytes per stored complex entry, vb = bytes per vector real."""
    cb = 2 * vb
    vec_m = Nt * Nm * vb
    spec_m = nfreq * Nm * cb
    fhat = nfreq * Nd * Nm * sb
    part = nfreq * nspan * Nd * cb
    dh = nfreq * Nd * cb
    return {
        "fft_r2c_m": vec_m + spec_m,
        "sbgemv_n": fhat + spec_m + part,
        "dside_h": part + dh,
        "sbgemv_c": fhat + dh + spec_m,
        "fft_c2r_m": spec_m + 2 * vec_m + vec_m,
    }


def measured_traffic(kernel, variant, storage="fp32"):
    """(HBM bytes per launch of `kernel` (variant id), summary path) from the committed
    rocprofv3 counter summary of that storage, or (None, None) when the summary is missing or
    was taken on a different kernel source."""
    import hashlib
    rel = os.path.join("profiles", "sbgemv_%s_nt420_nd100_nm65536_hbm_traffic.md" % storage)
    try:
        text = open(os.path.join(ROOT, rel)).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        data = json.loads(block)
        csrc = os.path.join(ROOT, "paper_2407_13066_amd", "csrc")
        src = hashlib.sha256(open(os.path.join(csrc, "sbgemv.hip"), "rb").read() +
                             open(os.path.join(csrc, "common.h"), "rb").read()).hexdigest()
        if src != data["source_sha256"]:
            return None, None
        return data["variants"]["%s/%d" % (kernel, variant)]["traffic_bytes"], \
            rel + " (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, scaled by a plain device copy)"
    except (OSError, IndexError, KeyError, ValueError):
        return None, None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return os.cpu_count() or 1


def oracle_H_columns(blocks, cols_by_dtype, noise_prec=1.0, prior_prec=1.0):
    """FP64 oracle H of the given input columns (the exact values the device saw), per input
    precision: {dtype name: [H(col) ...]}."""
    import oracle
    out = {}
    for name, cols in cols_by_dtype.items():
        out[name] = [oracle.apply_H(blocks, c.astype(np.float64), noise_prec, prior_prec) for c in cols]
    return out


def multi_rhs_benchmark(bt, blocks, op32, ks, h1_ms, storages=("f32", "bf16", "f64"), check_cols=(0, 7), op64=None,
                        h64_ms=None):
    """H applies with k stacked right-hand sides on the FP32-, BF16- and FP64-stored operator
    (matrix-core products): per-right-hand-side time against the single-vector H of the same
    storage (gain at that storage's accuracy), matrix-core throughput of the products, and
    the error against the FP64 oracle of columns ``check_cols`` at every k.

    Column r of a k-batch is the same vector for every k (counter-based generator), so the
    oracle H of each checked column is computed once per input precision."""
    import torch
    import synth
    Nt, Nd, Nm = blocks.shape
    cols = [c for c in check_cols if c < max(ks)]
    ncol = max(cols) + 1
    log("oracle H of columns %s (FP32 and FP64 inputs) for the multi-RHS errors" % cols)
    m32 = synth.vectors(ncol, Nt, Nm, synth.STREAM_M, dtype=np.float32)
    m64 = synth.vectors(ncol, Nt, Nm, synth.STREAM_M)
    refs = oracle_H_columns(blocks, {"f32": [m32[c] for c in cols], "f64": [m64[c] for c in cols]})
    out = {"checked_columns": cols}
    for storage in storages:
        if storage in ("f32", "f32split"):
            # f32split: the FP32-stored operator with its products on the BF16 matrix cores
            op = op32
            bt.btoep_set_gemm(op, storage == "f32split")
        elif storage == "f64" and op64 is not None:
            op = op64
        else:
            op = bt.btoep_create(blocks, storage)
            bt.btoep_autotune(op, reps=3)
        vn = np.float64 if storage == "f64" else np.float32
        ref = refs["f64" if storage == "f64" else "f32"]
        res = {}
        h1 = {"f32": h1_ms, "f32split": h1_ms, "f64": h64_ms}.get(storage)
        if h1 is None:
            # the single-vector H of this storage, the baseline of its gains
            m1 = torch.from_numpy(synth.vectors(1, Nt, Nm, synth.STREAM_M, dtype=vn)).cuda()
            o1 = torch.empty_like(m1)
            bt.btoep_apply_H(op, m1, 1.0, 1.0, out=o1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                bt.btoep_apply_H(op, m1, 1.0, 1.0, out=o1)
            torch.cuda.synchronize()
            h1 = (time.perf_counter() - t) * 1e3 / 5
            err1 = oracle_rel(o1[0], ref[0])
            res["k1"] = {"ms": round(h1, 3), "rel_err": err1}
            log("%s storage k=1: %.2f ms per H, rel err %.2e" % (storage, h1, err1))
            del m1, o1
        for k in ks:
            tune = None
            if storage != "f64":
                # matrix-core kernel variants for this k (the storage's mode as set)
                tune = bt.btoep_autotune_gemm(op, k, allow_split=False, reps=2)
                log("gemm autotune %s k=%d: N %s -> %d, C %s -> %d" % (
                    storage, k, list(tune["ms_n"].values())[0], tune["var_n"], list(tune["ms_c"].values())[0],
                    tune["var_c"]))
            M = torch.from_numpy(synth.vectors(k, Nt, Nm, synth.STREAM_M, dtype=vn)).cuda()
            HM = torch.empty_like(M)
            ws = torch.empty(bt.btoep_workspace_size(op, "H", k), dtype=torch.uint8, device="cuda")
            bt.btoep_apply_H(op, M, 1.0, 1.0, out=HM, ws=ws)
            torch.cuda.synchronize()
            bt.btoep_profile_enable(op, True)
            reps = 3
            t = time.perf_counter()
            for _ in range(reps):
                bt.btoep_apply_H(op, M, 1.0, 1.0, out=HM, ws=ws)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3 / reps
            prof = bt.btoep_profile_read(op)
            bt.btoep_profile_enable(op, False)
            flops = 8.0 * (Nt + 1) * Nd * Nm * k  # one product pass
            kern = {}
            for name in ("sbgemv_n", "sbgemv_c", "fft_r2c_m", "fft_c2r_m"):
                if name in prof:
                    avg = prof[name][1] / prof[name][0]
                    kern[name] = {"avg_ms": round(avg, 3)}
                    if name.startswith("sbgemv"):
                        kern[name]["TFLOPs"] = round(flops / (avg * 1e-3) / 1e12, 1)
            errs = {str(c): oracle_rel(HM[c], ref[i]) for i, c in enumerate(cols) if c < k}
            res["k%d" % k] = {"ms": round(ms, 3), "ms_per_rhs": round(ms / k, 4),
                              "gain_vs_k1": round(h1 / (ms / k), 2), "products": kern, "rel_err": errs}
            if tune is not None:
                res["k%d" % k]["gemm_autotune"] = tune
            if storage == "bf16":
                res["k%d" % k]["gain_vs_fp32_k1"] = round(h1_ms / (ms / k), 2)
            log("multi-RHS %s k=%d: %.2f ms (%.3f ms/RHS, x%.1f vs its k=1), rel err %s" % (
                storage, k, ms, ms / k, h1 / (ms / k), {c: "%.1e" % e for c, e in errs.items()}))
            del M, HM, ws
            torch.cuda.empty_cache()
        res["tolerance"] = {"f64": 1e-12, "f32": 1e-5, "f32split": 1e-5, "bf16": 3e-3}[storage]
        out[storage] = res
        if op is op32:
            bt.btoep_set_gemm(op, False)
        elif op is not op64:
            op.destroy()
    return out


def oracle_rel(dev_vec, ref):
    """Relative l2 error of a device vector against an FP64 oracle vector."""
    return float(np.linalg.norm(dev_vec.double().cpu().numpy() - ref) / np.linalg.norm(ref))


def serving_benchmark(bt, n_req, rates, seed=13066, n_cap=200, check=True):
    """Continuous-batching server over the three resident serving operators (FP32 storage for
    the applies, plus an FP64 copy of each for the refinement residuals of CG): a sustained
    saturating run measures capacity, then Poisson arrivals at fractions of it give p50 / p99
    latency and right-hand-side applies per second.  Request mix: kind uniform over
    F / FT / H / CG, operator uniform, k uniform in 1..16; H and CG use noise_prec = 1e4,
    prior_prec = 1e-3; CG right-hand sides are b = 1e4 F^T y (the inverse problem's form, y ~
    N(0,1) data vectors, formed in FP64), and a CG request stops once its true FP64 residual
    ||b - H x|| <= 1e-6 ||b|| (FP32 inner iterations, FP64 refinement; at most 500 inner
    iterations).  Every CG request's true residual is reported; a few requests of each kind are
    rerun alone and compared, and CG answers on the two smaller operators are checked with the
    FP64 oracle's H."""
    import torch
    import synth
    from paper_2407_13066_amd.serving import GpuExecutor, Request, Server, percentile

    shapes = synth.WORKLOADS["serving-3ops"]["ops"]
    ops, ops_hi = {}, {}
    for i, (Nt, Nd, Nm) in enumerate(shapes):
        blocks = synth.blocks(Nt, Nd, Nm, Nt / 7.0, stream=10 + i)
        ops["ABC"[i]] = bt.btoep_create(blocks, "f32")
        ops_hi["ABC"[i]] = bt.btoep_create(blocks, "f64")
        del blocks
    log("serving operators: " + ", ".join("%s %s %.2f GB (+ %.2f GB FP64)" % (
        n, shapes[i], ops[n].info["fhat_bytes"] / 1e9, ops_hi[n].info["fhat_bytes"] / 1e9)
        for i, n in enumerate("ABC")))
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    kinds = ("F", "FT", "H", "CG")
    noise, prior, rtol = 1e4, 1e-3, 1e-6

    # request inputs are read-only: every request takes k consecutive vectors of a resident pool
    # of 32 per (operator, input type), at a random offset, so thousands of requests need no
    # more device memory than the pool
    npool = 32
    pool = {}
    for name, op in ops.items():
        pool[(name, "m")] = torch.randn((npool, op.Nt, op.Nm), generator=gen, device="cuda")
        pool[(name, "d")] = torch.randn((npool, op.Nt, op.Nd), generator=gen, device="cuda")
        # inverse-problem right-hand sides b = sigma^-2 F^T y (y data vectors), in FP64
        y = torch.randn((npool, op.Nt, op.Nd), generator=gen, device="cuda", dtype=torch.float64)
        pool[(name, "b")] = bt.btoep_apply_FT(ops_hi[name], y).mul_(noise)
        del y

    def make(rid):
        name = "ABC"[int(rng.integers(3))]
        kind = kinds[int(rng.integers(4))]
        k = int(rng.integers(1, 17))
        o = int(rng.integers(0, npool - k + 1))
        x = pool[(name, {"CG": "b", "FT": "d"}.get(kind, "m"))][o:o + k]
        return Request(rid=rid, op=name, kind=kind, x=x, noise_prec=noise, prior_prec=prior, rtol=rtol,
                       max_iter=500, inner_rtol=1e-6)

    def release(done, keep=()):
        for r in done:
            if r not in keep:
                r.out = None

    # graphs for every batch shape the server can form, captured before any timing
    ex_graph = GpuExecutor(ops, n_streams=2, max_batch=32, use_graphs=True, ops_hi=ops_hi)
    ex_eager = GpuExecutor(ops, n_streams=2, max_batch=32, use_graphs=False, ops_hi=ops_hi)
    tuned = ex_graph.autotune(reps=2)   # the operators are shared: this tunes both executors
    log("serving autotune (matrix cores, per bucket: forward / adjoint variant, split): " + "; ".join(
        "%s %s" % (name, " ".join("k%d %d/%d%s" % (k, t["var_n"], t["var_c"], "s" if t["split"] else "")
                                  for k, t in res["gemm"].items()))
        for (name, level), res in tuned.items() if "gemm" in res))
    t0 = time.perf_counter()
    pipes = [(n, p, nz, pr) for n in "ABC" for p, nz, pr in (("F", 0.0, 0.0), ("FT", 0.0, 0.0), ("H", noise, prior))]
    ex_graph.prepare_graphs(pipes, range(1, 33))
    ex_graph.prepare_graphs([(n, "H", noise, prior) for n in "ABC"], range(1, 33), hi=True)
    capture_s = time.perf_counter() - t0
    log("captured %d serving graphs in %.2f s" % (len(ex_graph.graphs), capture_s))
    launch_cost = graph_launch_benchmark(bt, ops, ex_graph, ex_eager)

    def summary(done, wall, srv=None):
        lat = [r.latency * 1e3 for r in done]
        res = {"requests": len(done), "wall_s": round(wall, 3),
               "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
               "requests_per_s": round(len(done) / wall, 2)}
        for kind in kinds:
            lk = [r.latency * 1e3 for r in done if r.kind == kind]
            if lk:
                res["p50_p99_ms_" + kind] = [round(percentile(lk, 50), 2), round(percentile(lk, 99), 2)]
        cg = [r for r in done if r.kind == "CG"]
        if cg:
            res["cg"] = {"requests": len(cg), "unconverged": sum(1 for r in cg if not r.converged),
                         "max_true_rel_residual": max(max(r.rel_residual or [float("inf")]) for r in cg),
                         "rtol": rtol, "inner_iters_mean": round(float(np.mean([r.iters for r in cg])), 1),
                         "refinement_steps_mean": round(float(np.mean([r.outer for r in cg])), 2)}
        if srv is not None:
            rhs = sum(srv.rhs_applies.values())
            res.update({"rhs_applies_per_s": round(rhs / wall, 1), "rhs_applies_by_pipeline": dict(srv.rhs_applies),
                        "launches": srv.launches, "peak_request_GB": round(srv.peak_used / 1e9, 2)})
        return res

    def keep_few():
        """on_done hook: keep the answers the checks rerun (the first 6 applies and the first 3
        CG solves on operators A and B), drop the rest as requests complete."""
        kept = {"apply": 0, "cg": 0}

        def on_done(r):
            key = "cg" if r.kind == "CG" else "apply"
            if kept[key] < (3 if key == "cg" else 6) and not (r.kind == "CG" and r.op == "C"):
                kept[key] += 1
            else:
                r.out = None
        return on_done

    def run(arrivals, ex=ex_graph, label=""):
        srv = Server(ex, hbm_budget=64 << 30, max_batch=32, n_streams=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = [t0]

        def progress(n_done, n_all):
            if time.perf_counter() - last[0] > 20.0:
                last[0] = time.perf_counter()
                log("  serving %s: %d of %d requests done" % (label, n_done, n_all))
        done = srv.run(arrivals, t0=t0, timeout=1500, progress=progress, on_done=keep_few())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return srv, done, summary(done, wall, srv)

    # capacity: a saturating run (every request queued at once), throughput taken between the
    # 10th and the 90th percentile completion, so neither the ramp-up nor the drain counts
    sat = [(0.0, make(i)) for i in range(n_cap)]
    _, done_cap, cap = run(sat, label="capacity")
    release(done_cap)
    t_done = sorted(r.t_done for r in done_cap)
    i10, i90 = int(0.1 * len(t_done)), int(0.9 * len(t_done)) - 1
    capacity = (i90 - i10) / (t_done[i90] - t_done[i10])
    log("serving capacity (saturating run of %d requests, 10-90%% window): %.1f requests/s" % (n_cap, capacity))
    out = {"operators": {n: list(shapes[i]) for i, n in enumerate("ABC")}, "storage": "c64 (+ c128 for CG refinement)",
           "gemm_autotune": {name: {"k%d" % k: {"var_n": t["var_n"], "var_c": t["var_c"], "split_bf16": t["split"]}
                                    for k, t in res["gemm"].items()}
                             for (name, level), res in tuned.items() if "gemm" in res},
           "graphs": {"count": len(ex_graph.graphs), "capture_s": round(capture_s, 2), "per_apply_ms": launch_cost},
           "capacity_requests_per_s": round(capacity, 2),
           "capacity_run": dict(cap, window="10th-90th percentile completions"), "rates": {}}
    last = None
    for frac in rates:
        lam = frac * capacity
        t, arrivals = 0.0, []
        for i in range(n_req):
            t += float(rng.exponential(1.0 / lam))
            arrivals.append((t, make(1000 * (1 + len(out["rates"])) + i)))
        srv, done, res = run(arrivals, label="%.2fx" % frac)
        out["rates"]["%.2fx" % frac] = res
        log("serving at %.2fx capacity: p50 %.2f ms, p99 %.2f ms, %.0f RHS-applies/s, CG max true residual %s" % (
            frac, res["p50_ms"], res["p99_ms"], res["rhs_applies_per_s"],
            "%.2e" % res["cg"]["max_true_rel_residual"] if "cg" in res else "-"))
        if last is None and n_req <= 400:
            # the same arrivals with batches launched kernel by kernel instead of graph replays
            _, done_e, res_e = run([(t, Request(rid=r.rid, op=r.op, kind=r.kind, x=r.x, noise_prec=r.noise_prec,
                                                prior_prec=r.prior_prec, rtol=r.rtol, max_iter=r.max_iter,
                                                inner_rtol=r.inner_rtol)) for t, r in arrivals], ex=ex_eager,
                                   label="no graphs")
            release(done_e)
            out["rates"]["%.2fx_no_graphs" % frac] = res_e
            log("  same arrivals without graphs: p50 %.2f ms, p99 %.2f ms" % (res_e["p50_ms"], res_e["p99_ms"]))
        if last is not None:
            release(last)
        last = done
        torch.cuda.empty_cache()
    if check:
        out["checks"] = serving_checks(bt, ops, ops_hi, last, shapes, noise, prior, rtol)
    ex_graph.close()
    ex_eager.close()
    for op in list(ops.values()) + list(ops_hi.values()):
        op.destroy()
    return out


def serving_checks(bt, ops, ops_hi, done, shapes, noise, prior, rtol):
    """Requests of the last run rerun alone (F / FT / H: same operator and scalars; CG: the
    same refined stepwise solve driven one request at a time) and compared with their answers
    from the mix; CG answers on operators A and B checked with the FP64 oracle's H."""
    import torch
    import oracle
    import synth
    from tests.gpu_helpers import stepwise_cg
    worst, worst_cg, cg_oracle = 0.0, 0.0, []
    picked = [r for r in done if r.out is not None]
    for req in picked:
        op = ops[req.op]
        if req.kind == "CG":
            x, _, _ = stepwise_cg(bt, op, ops_hi[req.op], req.x, req.rtol, req.noise_prec, req.prior_prec,
                                  inner_rtol=req.inner_rtol, max_iter=req.max_iter, max_outer=req.max_outer)
            torch.cuda.synchronize()
            a, b = req.out, x
            worst_cg = max(worst_cg, float(torch.linalg.norm(a - b) / torch.linalg.norm(b)))
            i = "ABC".index(req.op)
            Nt, Nd, Nm = shapes[i]
            blocks = synth.blocks(Nt, Nd, Nm, Nt / 7.0, stream=10 + i)
            bh, xh = req.x[0].cpu().numpy(), req.out[0].cpu().numpy()
            res = np.linalg.norm(bh - oracle.apply_H(blocks, xh, noise, prior)) / np.linalg.norm(bh)
            cg_oracle.append({"op": req.op, "k": req.k, "oracle_true_rel_residual_col0": float(res),
                              "reported": req.rel_residual[0]})
            del blocks
            continue
        ref = {"F": lambda: bt.btoep_apply_F(op, req.x), "FT": lambda: bt.btoep_apply_FT(op, req.x),
               "H": lambda: bt.btoep_apply_H(op, req.x, req.noise_prec, req.prior_prec)}[req.kind]()
        torch.cuda.synchronize()
        a, b = req.out.double(), ref.double()
        worst = max(worst, float(torch.linalg.norm(a - b) / torch.linalg.norm(b)))
    log("serving checks: applies mixed vs alone %.2e, CG mixed vs alone %.2e, CG oracle residuals %s" % (
        worst, worst_cg, [round(c["oracle_true_rel_residual_col0"], 9) for c in cg_oracle]))
    return {"applies_mixed_vs_alone_max_rel_diff": worst, "cg_mixed_vs_alone_max_rel_diff": worst_cg,
            "cg_oracle": cg_oracle,
            "note": "CG answers from the mix and alone both meet rtol on the true residual; they differ by at most "
                    "~2 rtol cond(H) relative (cond(H) ~1e10-1e13 here), mostly in components of the null space of F"}


def graph_launch_benchmark(bt, ops, ex_graph, ex_eager, reps=200):
    """Per-apply time of back-to-back applies on one stream: pointer-array applies launched
    kernel by kernel, against replays of the captured graph with its address table rewritten
    every replay (as the server does) and without (as a solver's iteration does)."""
    import torch
    out = {}
    for name, op in ops.items():
        for pipe, k in (("H", 1), ("H", 8), ("F", 1)):
            n_in = op.Nd if pipe == "FT" else op.Nm
            n_out = op.Nd if pipe == "F" else op.Nm
            x = torch.randn((k, op.Nt, n_in), device="cuda")
            y = torch.empty((k, op.Nt, n_out), device="cuda")
            ins = [x[r].data_ptr() for r in range(k)]
            outs = [y[r].data_ptr() for r in range(k)]
            noise, prior = (1e4, 1e-3) if pipe == "H" else (0.0, 0.0)
            st = ex_graph.streams[0]
            g = ex_graph._graph(name, pipe, noise, prior, k, 0)
            res = {}
            for mode in ("eager", "graph", "graph_same_vectors"):
                def once():
                    if mode == "graph":
                        g.launch(ins, outs, stream=st)
                    elif mode == "graph_same_vectors":
                        g.launch(stream=st)
                    else:
                        bt.btoep_apply_batched_ptrs(op, pipe, ins, outs, noise, prior, ws=ex_eager.ws[(name, "lo")][0],
                                                    stream=st)
                for _ in range(5):
                    once()
                torch.cuda.synchronize()
                reps_op = max(10, min(reps, int(2e9 / max(op.info["fhat_bytes"], 1))))
                t0 = time.perf_counter()
                for _ in range(reps_op):
                    once()
                torch.cuda.synchronize()
                res[mode] = round((time.perf_counter() - t0) * 1e3 / reps_op, 4)
            out["%s_%s_k%d" % (name, pipe, k)] = res
            log("apply %s %s k=%d: %.4f ms eager, %.4f ms graph, %.4f ms graph on the same vectors" % (
                name, pipe, k, res["eager"], res["graph"], res["graph_same_vectors"]))
            del x, y
    return out


def paper_shapes_benchmark(bt):
    """The paper's single-GPU shapes in FP64 (its precision), as context: Nt=2000, Nd=7,
    Nm=60000 (its step breakdown), Nt=2000, Nd=100, Nm=4000 (largest of its Nm x Nd sweep) and
    Nm=800, Nd=100, Nt in {1000, 10000} (ends of its Nt sweep; Nt = 10000 needs four-step
    transforms).  F and F^T times after autotuning (which also picks the transform mode), and
    the effective bandwidth of F: operator + m + spectra written and read + d, per F time."""
    import torch
    import synth
    out = []
    for Nt, Nd, Nm in ((2000, 7, 60000), (2000, 100, 4000), (1000, 100, 800), (10000, 100, 800)):
        blocks = synth.blocks(Nt, Nd, Nm, Nt / 7.0, stream=20)
        op = bt.btoep_create(blocks, "f64")
        del blocks
        tune = bt.btoep_autotune(op, reps=3)
        m = torch.randn((Nt, Nm), dtype=torch.float64, device="cuda")
        d = torch.randn((Nt, Nd), dtype=torch.float64, device="cuda")

        def per_call(fn, reps=10):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) * 1e3 / reps

        f_ms = per_call(lambda: bt.btoep_apply_F(op, m))
        ft_ms = per_call(lambda: bt.btoep_apply_FT(op, d))
        nf = op.info["nfreq"]
        f_bytes = op.info["fhat_bytes"] + 8 * Nt * Nm + 2 * 16 * nf * Nm + 8 * Nt * Nd
        gbs = f_bytes / (f_ms * 1e-3) / 1e9
        res = {"Nt": Nt, "Nd": Nd, "Nm": Nm, "storage": "c128", "fhat_GB": round(op.info["fhat_bytes"] / 1e9, 2),
               "F_ms": round(f_ms, 3), "FT_ms": round(ft_ms, 3), "F_GBs": round(gbs, 1),
               "F_pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 1),
               "transforms": "four-step" if tune["fft_four_step"] else "single-pass",
               "transform_pair_ms": tune["ms_fft"]}
        log("paper shape Nt=%d Nd=%d Nm=%d FP64: F %.3f ms (%.0f GB/s), F^T %.3f ms, %s transforms" % (
            Nt, Nd, Nm, f_ms, gbs, ft_ms, res["transforms"]))
        out.append(res)
        op.destroy()
        del m, d
        torch.cuda.empty_cache()
    return out


def appendix_benchmark(bt):
    """The paper's appendix comparison in FP64: its alternate local matvec (SOTI products, then
    sums over block rows / columns) against the frequency-outer products, at the two shapes the
    appendix reports (Nt=2000 with Nd=7, Nm=40000 and with Nd=100, Nm=4000).  Mode 0 writes the
    products to a matrix-sized buffer and reduces them in a second kernel, as the appendix does;
    mode 1 forms them inside the reduction."""
    import torch
    import synth
    out = []
    for Nt, Nd, Nm in ((2000, 7, 40000), (2000, 100, 4000)):
        blocks = synth.blocks(Nt, Nd, Nm, Nt / 7.0, stream=21)
        op = bt.btoep_create(blocks, "f64")
        del blocks
        bt.btoep_autotune(op, reps=3)
        m = torch.randn((Nt, Nm), dtype=torch.float64, device="cuda")
        d = torch.randn((Nt, Nd), dtype=torch.float64, device="cuda")

        def per_call(fn, reps=10):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) * 1e3 / reps

        res = {"Nt": Nt, "Nd": Nd, "Nm": Nm, "storage": "c128",
               "main_F_ms": round(per_call(lambda: bt.btoep_apply_F(op, m)), 3),
               "main_FT_ms": round(per_call(lambda: bt.btoep_apply_FT(op, d)), 3)}
        for mode in (1, 0):
            bt.btoep_alt_prepare(op, mode)
            res["alt%d_F_ms" % mode] = round(per_call(lambda: bt.btoep_alt_apply(op, "F", m, mode=mode)), 3)
            res["alt%d_FT_ms" % mode] = round(per_call(lambda: bt.btoep_alt_apply(op, "FT", d, mode=mode)), 3)
        log("appendix form Nt=%d Nd=%d Nm=%d FP64: F main %.3f / fused %.3f / two-kernel %.3f ms; "
            "F^T %.3f / %.3f / %.3f ms" % (Nt, Nd, Nm, res["main_F_ms"], res["alt1_F_ms"], res["alt0_F_ms"],
                                            res["main_FT_ms"], res["alt1_FT_ms"], res["alt0_FT_ms"]))
        out.append(res)
        op.destroy()
        del m, d
        torch.cuda.empty_cache()
    return out


def setup_benchmark(bt, blocks, storage, host_s):
    """Setup of the stored operator (transform of every block series, Alg. 1 on one device) from
    device-resident FP64 blocks, given as the first block column and as the last block row; the
    host-input setup time of the main operator (PCIe-bound staging included) for context.
    Algorithmic bytes: the FP64 blocks read once plus the stored spectra written once."""
    import torch
    Nt, Nd, Nm = blocks.shape
    dev_blocks = torch.from_numpy(blocks).cuda()
    op = bt.btoep_create_empty(Nt, Nd, Nm, storage)
    sb = {"f64": 16, "f32": 8, "bf16": 4}[storage]
    nbytes = blocks.nbytes + op.info["nfreq"] * Nd * Nm * sb
    out = {"host_create_s": round(host_s, 3), "algorithmic_GB": round(nbytes / 1e9, 2)}
    for order, src in (("column", dev_blocks), ("last_row", None)):
        if src is None:
            src = torch.flip(dev_blocks, [0])
            del dev_blocks
        bt.btoep_set_blocks(op, 0, 0, src, order=order)  # warm-up (returns when done)
        t = time.perf_counter()
        bt.btoep_set_blocks(op, 0, 0, src, order=order)
        ms = (time.perf_counter() - t) * 1e3
        out["device_%s_ms" % order] = round(ms, 2)
        out["device_%s_GBs" % order] = round(nbytes / (ms * 1e-3) / 1e9, 1)
        del src
    log("setup: host %.2f s; device block column %.1f ms (%.0f GB/s), last block row %.1f ms" % (
        host_s, out["device_column_ms"], out["device_column_GBs"], out["device_last_row_ms"]))
    op.destroy()
    torch.cuda.empty_cache()
    return out


def cg_benchmark(bt):
    """Inverse-problem CG: H = sigma^-2 F^T F + alpha I with sigma = 1e-2, alpha = 1e-3 on
    Nt=256, Nd=64, Nm=16384 (blocks N(0,1) exp(-k/(Nt/7))), d = F m_true + N(0, sigma^2),
    b = sigma^-2 F^T d, to a true relative residual of 1e-8: all-FP64 CG against FP32-inner
    CG with FP64 iterative refinement, each with inner iterations replayed from a graph and
    launched kernel by kernel.  b is formed with the FP64 operator on the device."""
    import torch
    import synth
    w = synth.WORKLOADS["cg-nt256-nd64-nm16384"]
    Nt, Nd, Nm = w["Nt"], w["Nd"], w["Nm"]
    sigma, alpha = w["sigma"], w["alpha"]
    blocks = synth.blocks(Nt, Nd, Nm, w["tau"])
    hi = bt.btoep_create(blocks, "f64")
    lo = bt.btoep_create(blocks, "f32")
    del blocks
    for op in (hi, lo):
        bt.btoep_autotune(op, reps=3)
    m_true = torch.from_numpy(synth.vectors(1, Nt, Nm, synth.STREAM_MTRUE)).cuda()
    noise = torch.from_numpy(synth.vectors(1, Nt, Nd, synth.STREAM_NOISE)).cuda()
    dobs = bt.btoep_apply_F(hi, m_true) + sigma * noise
    b = bt.btoep_apply_FT(hi, dobs).mul_(sigma ** -2)
    out = {"workload": "cg-nt256-nd64-nm16384", "sigma": sigma, "alpha": alpha, "rtol": w["rtol"]}
    sols = {}
    for name, op_lo, op_hi, inner_rtol in (("fp64", hi, None, 1e-9), ("fp32_refined", lo, hi, 1e-5)):
        for use_graph in (True, False):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, res = bt.btoep_cg_solve(op_lo, op_hi, b, x, sigma ** -2, alpha, rtol=w["rtol"], max_outer=20,
                                        max_inner=5000, inner_rtol=inner_rtol, check_every=8, use_graph=use_graph)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            r = res[0]
            key = name + ("" if use_graph else "_no_graph")
            out[key] = {"status": st, "seconds": round(sec, 4), "inner_iters": r["inner_iters"],
                        "outer_iters": r["outer_iters"], "matvecs": r["matvecs"],
                        "true_rel_residual": r["rel_residual"],
                        "ms_per_matvec": round(sec * 1e3 / max(r["matvecs"], 1), 4)}
            sols[key] = x
            log("cg %s: %.3f s, %d inner + %d outer, true rel residual %.2e" % (
                key, sec, r["inner_iters"], r["outer_iters"], r["rel_residual"]))
    # BF16-stored inner operator (relative storage error ~2e-3) inside FP64 refinement: a
    # bounded run (at most 8 refinement steps of 400 inner iterations), outcome as measured
    lo16 = bt.btoep_create(synth.blocks(Nt, Nd, Nm, w["tau"]), "bf16")
    bt.btoep_autotune(lo16, reps=3)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, res = bt.btoep_cg_solve(lo16, hi, b, x, sigma ** -2, alpha, rtol=w["rtol"], max_outer=8, max_inner=400,
                                inner_rtol=1e-2, check_every=8)
    torch.cuda.synchronize()
    r = res[0]
    out["bf16_refined"] = {"status": st, "converged": bool(r["converged"]), "seconds": round(time.perf_counter() - t0, 3),
                           "inner_iters": r["inner_iters"], "outer_iters": r["outer_iters"],
                           "true_rel_residual": r["rel_residual"],
                           "inner_rtol": 1e-2}
    log("cg bf16_refined: status %d, %d inner + %d outer, true rel residual %.2e" % (
        st, r["inner_iters"], r["outer_iters"], r["rel_residual"]))
    lo16.destroy()
    del x
    # the two solutions agree in the data space (null-space parts are not determined)
    Fd = bt.btoep_apply_F(hi, sols["fp32_refined"] - sols["fp64"])
    out["data_space_rel_diff"] = float(torch.linalg.norm(Fd) / torch.linalg.norm(bt.btoep_apply_F(hi, sols["fp64"])))
    out["graph_equals_no_graph"] = bool(torch.equal(sols["fp64"], sols["fp64_no_graph"]) and
                                        torch.equal(sols["fp32_refined"], sols["fp32_refined_no_graph"]))
    out["speedup_refined_vs_fp64"] = round(out["fp64"]["seconds"] / out["fp32_refined"]["seconds"], 2)
    hi.destroy()
    lo.destroy()
    return out


def small_case(bt, calls=50):
    """The small FP64 case (Nt=32, Nd=16, Nm=64; 0.5 MB operator, cache-resident): microseconds
    per F, F^T and H call (median over `calls` calls, each between HIP events on the launch
    stream), launched directly and as a graph replay on the same vectors, the full-vector error
    against the FP64 oracle, and the oracle's own time per call on the host."""
    import torch
    import oracle
    import synth
    w = synth.WORKLOADS["fp64-small"]
    Nt, Nd, Nm = w["Nt"], w["Nd"], w["Nm"]
    blocks = synth.blocks(Nt, Nd, Nm, w["tau"])
    op = bt.btoep_create(blocks, "f64")
    m = synth.vectors(1, Nt, Nm, synth.STREAM_M)
    d = synth.vectors(1, Nt, Nd, synth.STREAM_D)
    md, dd = torch.from_numpy(m).cuda(), torch.from_numpy(d).cuda()
    st = torch.cuda.Stream()
    ref = {"F": oracle.apply_F(blocks, m), "FT": oracle.apply_FT(blocks, d), "H": oracle.apply_H(blocks, m, 1.0, 1.0)}
    res = {"workload": "fp64-small", "Nt": Nt, "Nd": Nd, "Nm": Nm, "fhat_MB": round(op.info["fhat_bytes"] / 1e6, 3),
           "calls": calls}
    for which in ("F", "FT", "H"):
        x = dd if which == "FT" else md
        y = torch.empty((1, Nt, Nm if which != "F" else Nd), dtype=torch.float64, device="cuda")
        ws = torch.empty(bt.btoep_workspace_size(op, which, 1), dtype=torch.uint8, device="cuda")
        g = bt.ApplyGraph(op, which, 1, 1.0, 1.0, ws=ws)
        g.launch([x.data_ptr()], [y.data_ptr()], stream=st)

        def direct():
            bt.btoep_apply_batched_ptrs(op, which, [x.data_ptr()], [y.data_ptr()], 1.0, 1.0, ws=ws, stream=st)

        def replay():
            g.launch(stream=st)
        entry = {}
        for name, fn in (("direct", direct), ("graph", replay)):
            for _ in range(5):
                fn()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
            with torch.cuda.stream(st):
                for a, b in ev:
                    a.record(st)
                    fn()
                    b.record(st)
            st.synchronize()
            entry[name + "_us"] = round(1e3 * float(np.median([a.elapsed_time(b) for a, b in ev])), 2)
        direct()
        st.synchronize()
        entry["rel_err"] = oracle.rel_l2(y.cpu().numpy()[0], ref[which][0])
        g.destroy()
        res[which] = entry
    t = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.apply_H(blocks, m, 1.0, 1.0)
        t.append(time.perf_counter() - t0)
    res["oracle_H_us"] = round(1e6 * float(np.median(t)), 1)
    res["tolerance"] = 1e-12
    op.destroy()
    log("small FP64 case: " + ", ".join("%s %.1f us direct / %.1f us graph (rel err %.1e)" % (
        k, res[k]["direct_us"], res[k]["graph_us"], res[k]["rel_err"]) for k in ("F", "FT", "H")) +
        "; oracle H %.0f us" % res["oracle_H_us"])
    return res


def time_H(bt, op, m, out, ws, stream, steps, warmup, noise_prec, prior_prec):
    """Warm-up, then `steps` H applications bracketed by device synchronisation, with per-kernel
    HIP events on the launch stream.  Returns (ms per H, {kernel: (launches, total ms)})."""
    import torch
    for _ in range(warmup):
        bt.btoep_apply_H(op, m, noise_prec, prior_prec, out=out, ws=ws, stream=stream)
    torch.cuda.synchronize()
    bt.btoep_profile_enable(op, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bt.btoep_apply_H(op, m, noise_prec, prior_prec, out=out, ws=ws, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = bt.btoep_profile_read(op)
    bt.btoep_profile_enable(op, False)
    return (t1 - t0) * 1e3 / steps, kern


def roofline_block(kern, ab, sb, tune):
    """Roofline of the dominant kernel of an H: algorithmic bytes per launch / mean launch time
    (HIP events), with the HBM traffic of that kernel from the committed counter summary."""
    dom = max(kern.items(), key=lambda kv: kv[1][1])[0]
    dom_avg_s = kern[dom][1] / kern[dom][0] * 1e-3
    achieved = ab[dom] / dom_avg_s / 1e9
    storage = {16: "fp64", 8: "fp32", 4: "bf16"}[sb]
    traffic, src = None, None
    if dom in ("sbgemv_n", "sbgemv_c"):
        traffic, src = measured_traffic(dom, tune["var_n"] if dom == "sbgemv_n" else tune["var_c"], storage)
    return {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes": ab[dom], "avg_launch_ms": round(
                dom_avg_s * 1e3, 4), "traffic": traffic,
            "traffic_GBs": round(traffic / dom_avg_s / 1e9, 1) if traffic else None,
            "traffic_source": src}


def kernel_table(kern, ab):
    out = {}
    for name, (n, tot) in kern.items():
        avg = tot / max(n, 1)
        kb = ab.get(name)
        out[name] = {"launches": n, "avg_ms": round(avg, 4),
                     "algorithmic_GBs": round(kb / (avg * 1e-3) / 1e9, 1) if kb else None,
                     "pct_hbm_peak": round(100 * kb / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 1) if kb else None}
    return out


def headline_errors(bt, op, blocks, m, d, ws, stream, noise_prec, prior_prec, Hm):
    """Errors against the FP64 oracle: F m and F^T d over the full vectors, H m on 64 sampled
    entries (the oracle's full F m, then sampled entries of F^T)."""
    import torch
    import oracle
    rng = np.random.default_rng(7)
    Nt, Nd, Nm = blocks.shape
    Fm = bt.btoep_apply_F(op, m, ws=ws, stream=stream)
    FTd = bt.btoep_apply_FT(op, d, ws=ws, stream=stream)
    torch.cuda.synchronize()
    mh = m.double().cpu().numpy()  # the input the device saw
    dh = d.double().cpu().numpy()
    Fm_ref = oracle.apply_F(blocks, mh)
    FTd_ref = oracle.apply_FT(blocks, dh)
    idxH = [(int(rng.integers(Nt)), int(rng.integers(Nm))) for _ in range(64)]
    ftd = oracle.entries_FT(blocks, noise_prec * Fm_ref, idxH)
    Hs_ref = np.array([ftd[n] + prior_prec * mh[j, p] for n, (j, p) in enumerate(idxH)])
    Hm_h = Hm.double().cpu().numpy()
    Hs = np.array([Hm_h[j, p] for (j, p) in idxH])
    return {"F_full": oracle.rel_l2(Fm.double().cpu().numpy(), Fm_ref),
            "FT_full": oracle.rel_l2(FTd.double().cpu().numpy(), FTd_ref),
            "H_sampled64": oracle.rel_l2(Hs, Hs_ref)}


def cpu_baseline(blocks, m_host, noise_prec, prior_prec, sample_cols, one_thread_cols=2048):
    """The FP64 oracle's H timed on the host: all the cores this process may use (BLAS threads),
    on ``sample_cols`` parameter columns, and one thread on ``one_thread_cols`` columns; both
    scaled to the full Nm (the oracle's cost is linear in Nm)."""
    import oracle
    Nt, Nd, Nm = blocks.shape

    def timed(ncol, min_s):
        sb = blocks if ncol == Nm else np.ascontiguousarray(blocks[:, :, :ncol])
        ms_ = m_host if ncol == Nm else np.ascontiguousarray(m_host[:, :ncol])
        runs, t = 0, 0.0
        while runs < 3 and (runs == 0 or t < min_s):
            a = time.perf_counter()
            oracle.apply_H(sb, ms_, noise_prec, prior_prec)
            t += time.perf_counter() - a
            runs += 1
        return t / runs * (Nm / ncol), runs, t / runs

    ns = min(sample_cols, Nm)
    log("timing the CPU oracle on %d of %d parameter columns" % (ns, Nm))
    per, runs, each = timed(ns, 10.0)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    threads = blas_threads()
    res = {"value": round(1.0 / per, 5), "unit": "H matvecs/s", "cores": threads, "kind": "oracle",
           "host_cores_available": affinity,
           "sample": "FP64 oracle H (lag-outer block products, numpy matmul on %d BLAS threads) on %d of %d parameter "
                     "columns, same Nt and Nd, %d run(s), %.2f s each%s" % (
                         threads, ns, Nm, runs, each,
                         "" if ns == Nm else ", scaled x%.0f (cost is linear in Nm)" % (Nm / ns))}
    try:
        from threadpoolctl import threadpool_limits
        n1 = min(one_thread_cols, Nm)
        with threadpool_limits(limits=1):
            per1, runs1, each1 = timed(n1, 5.0)
        res["one_thread"] = {"value": round(1.0 / per1, 6), "unit": "H matvecs/s", "cores": 1,
                             "sample": "%d of %d parameter columns, %d run(s), %.2f s each, scaled x%.0f" % (
                                 n1, Nm, runs1, each1, Nm / n1)}
        log("cpu oracle: %.2f s per H on %d threads, %.1f s on one thread" % (per, threads, per1))
    except ImportError:
        pass
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (for scaling PMC byte counters)")
    ap.add_argument("--calibrate-read", action="store_true",
                    help="only measure the streaming-read and streaming-write rates of one 22 GB array (the memory system's ceilings)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline H timing (for profiler runs)")
    ap.add_argument("--f64-only", action="store_true",
                    help="only the FP64-storage H at the headline shape (for profiler runs)")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64-storage H at the headline shape")
    ap.add_argument("--multi-rhs", default="8,32,64",
                    help="comma-separated right-hand-side counts for the stacked-H measurement ('' skips it)")
    ap.add_argument("--serving-requests", type=int, default=150,
                    help="requests per arrival rate in the serving run (0 skips it)")
    ap.add_argument("--serving-rates", default="0.5,0.9",
                    help="arrival rates of the serving run, as fractions of the measured capacity")
    ap.add_argument("--serving-capacity-requests", type=int, default=200,
                    help="requests of the saturating run that measures serving capacity")
    ap.add_argument("--serving-only", action="store_true", help="only the serving measurement")
    ap.add_argument("--no-cg", action="store_true", help="skip the CG solve measurement")
    ap.add_argument("--no-paper-shapes", action="store_true", help="skip the paper-shape (FP64) context runs")
    ap.add_argument("--no-setup", action="store_true", help="skip the setup (block transform) measurement")
    ap.add_argument("--multi-rhs-storage", default="f32,f32split,bf16,f64",
                    help="operator storages of the multi-RHS measurement (comma separated)")
    ap.add_argument("--no-appendix", action="store_true",
                    help="skip the comparison with the paper's appendix (SOTI) matvec form")
    ap.add_argument("--cpu-sample-cols", type=int, default=65536,
                    help="parameter columns of the operator the CPU oracle is timed on")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (use --gpus 1)",
              file=sys.stderr)
        return 2

    import torch
    import synth
    import paper_2407_13066_amd as bt
    from paper_2407_13066_amd import build as btbuild

    if args.calibrate_copy:
        n = 1 << 30  # 4 GiB of float32 read and 4 GiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / 5
        print(json.dumps({"calibration": "device copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "ms": round(dt * 1e3, 4), "GBs_read_plus_write": round(8 * n / dt / 1e9, 1)}))
        return 0

    if not os.path.exists(bt.LIB_PATH):
        btbuild.build()
    bt.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calibrate_read:
        nbytes = 22 * 10 ** 9
        res = bt.btoep_read_bandwidth(nbytes, reps=5)
        wres = bt.btoep_write_bandwidth(nbytes, reps=5)
        print(json.dumps({"calibration": "streaming read", "bytes": nbytes, **res,
                          "write": {"calibration": "streaming write", "bytes": nbytes, **wres}}))
        return 0

    if args.serving_only:
        rates = tuple(float(v) for v in args.serving_rates.split(",") if v)
        res = serving_benchmark(bt, args.serving_requests, rates, n_cap=args.serving_capacity_requests)
        print(json.dumps({"measurement": "serving", "serving": res}), flush=True)
        return 0

    wname = "fp32-nt420-nd100-nm65536"
    w = synth.WORKLOADS[wname]
    Nt, Nd, Nm, tau = w["Nt"], w["Nd"], w["Nm"], w["tau"]
    noise_prec, prior_prec = w["noise_prec"], w["prior_prec"]
    log("generating blocks [%d][%d][%d] FP64 (%.1f GB)" % (Nt, Nd, Nm, Nt * Nd * Nm * 8 / 1e9))
    blocks = synth.blocks(Nt, Nd, Nm, tau)
    m_host = synth.vectors(1, Nt, Nm, synth.STREAM_M)[0]
    d_host = synth.vectors(1, Nt, Nd, synth.STREAM_D)[0]
    stream = torch.cuda.current_stream()
    result = {}
    op = None
    if not args.f64_only:
        log("creating operator (FP32 complex storage)")
        t_setup = time.perf_counter()
        op = bt.btoep_create(blocks, w["storage"])
        host_setup_s = time.perf_counter() - t_setup
        info = bt.btoep_query(op)
        log("operator: L=%d nfreq=%d fhat=%.2f GB" % (info["L"], info["nfreq"], info["fhat_bytes"] / 1e9))

        m = torch.from_numpy(m_host).to(dev, torch.float32)
        d = torch.from_numpy(d_host).to(dev, torch.float32)
        Hm = torch.empty_like(m)
        dd = torch.empty((Nt, Nd), dtype=torch.float32, device=dev)
        mt = torch.empty_like(m)

        tune = bt.btoep_autotune(op, reps=5, stream=stream)
        log("autotune: N %s -> %d, C %s -> %d; transforms %s ms (single-pass, four-step) -> %s" % (
            tune["ms_n"], tune["var_n"], tune["ms_c"], tune["var_c"], tune["ms_fft"],
            "four-step" if tune["fft_four_step"] else "single-pass"))
        ws = torch.empty(bt.btoep_workspace_size(op, "H", 1), dtype=torch.uint8, device=dev)  # after the mode choice

        ms_per_step, kern = time_H(bt, op, m, Hm, ws, stream, args.steps, args.warmup, noise_prec, prior_prec)
        log("H: %.3f ms/step" % ms_per_step)
        nspan = -(-Nm // 4096)  # spans of the N-direction product at this shape (4096 columns each)
        ab = algorithmic_bytes(Nt, Nd, Nm, info["nfreq"], nspan, 8, 4)
        H_bytes = sum(ab.values())
        result = {
            "metric": "H matvecs/s + HBM GB/s (% of peak) at stated rel err; serving p50/p99 ms",
            "value": round(1e3 / ms_per_step, 3),
            "unit": "H matvecs/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic (seeded N(0,1) exp(-k/60) blocks, N(0,1) vector)",
            "config": {"workload": wname, "Nt": Nt, "Nd": Nd, "Nm": Nm, "k": 1, "storage": "c64",
                       "noise_prec": noise_prec, "prior_prec": prior_prec},
            "H_algorithmic_GB": round(H_bytes / 1e9, 3),
            "H_GBs": round(H_bytes / (ms_per_step * 1e-3) / 1e9, 1),
            "H_pct_hbm_peak": round(100 * H_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 1),
            "kernels": kernel_table(kern, ab),
            "autotune": tune,
            "roofline": roofline_block(kern, ab, 8, tune),
        }
        if args.headline_only:
            print(json.dumps(result), flush=True)
            return 0

        def time_call(fn, reps=10):
            fn()
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - a) * 1e3 / reps

        result["F_ms"] = round(time_call(lambda: bt.btoep_apply_F(op, m, dd, ws=ws, stream=stream)), 4)
        result["FT_ms"] = round(time_call(lambda: bt.btoep_apply_FT(op, d, mt, ws=ws, stream=stream)), 4)
        log("F: %.3f ms, F^T: %.3f ms" % (result["F_ms"], result["FT_ms"]))
        if not args.no_check:
            log("checking F, F^T (full vectors) and H (sampled entries) against the FP64 oracle")
            result["rel_err"] = dict(headline_errors(bt, op, blocks, m, d, ws, stream, noise_prec, prior_prec, Hm),
                                     tolerance=1e-5)
            log("rel err %s" % {k: "%.2e" % v for k, v in result["rel_err"].items()})
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = cpu_baseline(blocks, m_host, noise_prec, prior_prec, args.cpu_sample_cols)
        del Hm, dd, mt, ws

    # the same H with the operator stored in FP64 (the paper's precision), FP64 vectors
    op64, h64_ms = None, None
    if not args.no_f64:
        log("creating operator (FP64 complex storage)")
        op64 = bt.btoep_create(blocks, "f64")
        info64 = bt.btoep_query(op64)
        tune64 = bt.btoep_autotune(op64, reps=3, stream=stream)
        m64 = torch.from_numpy(m_host).to(dev)
        d64 = torch.from_numpy(d_host).to(dev)
        Hm64 = torch.empty_like(m64)
        ws64 = torch.empty(bt.btoep_workspace_size(op64, "H", 1), dtype=torch.uint8, device=dev)
        steps64 = max(5, args.steps // 2)
        h64_ms, kern64 = time_H(bt, op64, m64, Hm64, ws64, stream, steps64, 2, noise_prec, prior_prec)
        ab64 = algorithmic_bytes(Nt, Nd, Nm, info64["nfreq"], -(-Nm // 2048), 16, 8)
        res64 = {"storage": "c128", "dtype": "f64", "steps": steps64, "ms_per_H": round(h64_ms, 4),
                 "H_per_s": round(1e3 / h64_ms, 3), "H_algorithmic_GB": round(sum(ab64.values()) / 1e9, 3),
                 "H_pct_hbm_peak": round(100 * sum(ab64.values()) / (h64_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1),
                 "kernels": kernel_table(kern64, ab64), "autotune": tune64,
                 "roofline": roofline_block(kern64, ab64, 16, tune64)}
        log("FP64 storage H: %.3f ms (%.1f%% of HBM peak over the whole H), roofline %s %.0f GB/s" % (
            h64_ms, res64["H_pct_hbm_peak"], res64["roofline"]["kernel"], res64["roofline"]["achieved"]))
        if args.f64_only:
            print(json.dumps({"measurement": "fp64 headline", "fp64_storage": res64}), flush=True)
            return 0
        if not args.no_check:
            res64["rel_err"] = dict(headline_errors(bt, op64, blocks, m64, d64, ws64, stream, noise_prec, prior_prec,
                                                    Hm64), tolerance=1e-12)
            log("FP64 rel err %s" % {k: "%.2e" % v for k, v in res64["rel_err"].items()})
        result["fp64_storage"] = res64
        del m64, d64, Hm64, ws64

    if args.multi_rhs:
        ks = [int(v) for v in args.multi_rhs.split(",") if v]
        result["multi_rhs"] = multi_rhs_benchmark(bt, blocks, op, ks, ms_per_step,
                                                  storages=[v for v in args.multi_rhs_storage.split(",") if v],
                                                  op64=op64, h64_ms=h64_ms)

    op.destroy()
    if op64 is not None:
        op64.destroy()
    torch.cuda.empty_cache()
    if not args.no_setup:
        result["setup"] = setup_benchmark(bt, blocks, w["storage"], host_setup_s)
    del blocks
    result["small_fp64"] = small_case(bt)
    if not args.no_cg:
        result["cg"] = cg_benchmark(bt)
        torch.cuda.empty_cache()
    if not args.no_paper_shapes:
        result["paper_shapes"] = paper_shapes_benchmark(bt)
        torch.cuda.empty_cache()
    if not args.no_appendix:
        result["appendix_form"] = appendix_benchmark(bt)
        torch.cuda.empty_cache()
    if args.serving_requests > 0:
        rates = tuple(float(v) for v in args.serving_rates.split(",") if v)
        result["serving"] = serving_benchmark(bt, args.serving_requests, rates, n_cap=args.serving_capacity_requests)

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
