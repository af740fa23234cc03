"""Benchmark: exact eps-join of 1,000,000 x 1,000,000 unit-norm vectors
(d = 128) with bf16 candidates on one GPU.

One step is the whole hot path over one batch of synthetic input already
resident in HBM: operand prep of R and S (norms, bf16 copies, residual
bounds), the matrix-core candidate pass with the fused margin-widened eps
filter, the float32 / float64 recheck of every candidate and the canonical
(i, j) ordering of the emitted pairs.  R and S are drawn from a 1,000-centre
Gaussian mixture on the sphere (sigma 0.05); eps is the lower median of the
exact 10th-neighbour distance of 256 seeded rows of R.  `value` is the
number of distance pairs in the join's domain (|R| |S|) per second of step
time.

Beside the headline the line carries: the plain fp32 join on the same input
(its (i, j) arrays compared with the timed result), the top-10 join of the
same relations, the featurise + self-join of 100,000 RGB patches (fp32
candidates as that workload states, and the exact fp16 variant), the E4M3
and bf16 top-32 of 50,000 queries against a 4,000,000 x 256 store, the
serving loop, and the float64 oracle on seeded rows (its time, and the
element-wise agreement of those rows with the timed result).

Prints one JSON line.  Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp8": 5000.0, "fp32": 157.3}
METRIC = "G distance-pairs/s for ε-join at exact pair set; p50/p99 query latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="bf16", choices=sorted(PEAK_TFLOPS), help="candidate format of the headline")
    ap.add_argument("--n", type=int, default=1000000, help="rows of R and of S (default: the full workload)")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: no fp32 comparison, top-10, histogram, store or serving legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-store", type=int, default=8000000, help="rows of the serving store")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="open-loop seconds per offered rate")
    ap.add_argument("--crossover", action="store_true",
                    help="instead of the headline step, sweep the histogram self-join size and time the CPU oracle "
                         "against the GPU join (device-resident and with the host transfers) (one JSON line)")
    ap.add_argument("--etl-only", action="store_true",
                    help="only the fused-store, index-pruned join, plan and crop legs (one JSON line)")
    ap.add_argument("--serving-only", action="store_true",
                    help="instead of the headline step, run the serving leg alone (profiling runs of the loop)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="copy this many MiB device-to-device first (scale for FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--histogram-headline", action="store_true",
                    help="instead of the headline step, time featurise + self-join of 100,000 patches (--prec, "
                         "default fp16 there) for profiling")
    ap.add_argument("--secondary", action="store_true",
                    help="instead of the headline step, time the unit-mixture eps and top-k joins (one JSON line)")
    ap.add_argument("--full-configs", action="store_true",
                    help="instead of the headline step, time the 1M x 1M d=128 joins (bf16 and fp32) and the "
                         "4M x 256 store with 50k top-32 queries (fp8 and bf16) at full size (one JSON line)")
    return ap.parse_args()


KERNEL_SOURCES = ["paper_1812_07607_amd/csrc/join_mfma.hip", "paper_1812_07607_amd/csrc/join_params.hpp",
                  "paper_1812_07607_amd/csrc/dl_internal.hpp"]
TRAFFIC_SUMMARY = {"bf16": "profiles/cand_kernel_bf16_eps_1m_d128_traffic.txt",
                   "fp16": "profiles/cand_kernel_fp16_selfjoin_100k_traffic.txt"}


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec, workload):
    """HBM bytes per launch of the contraction kernel from the committed
    rocprofv3 counter summary of this workload, if it was taken on the
    current kernel source (else None)."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY.get(prec, ""))
    if not os.path.isfile(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash() or vals.get("workload") != workload:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def timed_calls(ctx, fn, reps):
    """Stage times (ms per call, HIP events) of `reps` calls after one
    untimed call; returns (last result, per-stage dict)."""
    import torch
    r = fn()
    torch.cuda.synchronize()
    ctx.timing(reset=True)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    ctx.set_timing(False)
    st = ctx.timing(reset=True)
    rec = {k: round(v[0] / reps, 3) for k, v in st.items() if v[1]}
    rec["ms_per_call"] = round(wall * 1e3, 3)
    rec["contractions_per_call"] = round(st["contract"][1] / reps, 2)
    return r, rec


def rows_of(res, rows):
    """The pairs of an eps result whose i is one of `rows` (host int64 arrays
    i, j and float32 dist, in the result's (i, j) order)."""
    import numpy as np
    import torch
    gi = res.i.long() & 0xffffffff
    keep = torch.isin(gi, torch.from_numpy(np.asarray(rows, np.int64)).to(gi.device))
    return (gi[keep].cpu().numpy(), (res.j.long()[keep] & 0xffffffff).cpu().numpy(),
            res.dist[keep].cpu().numpy())


def cpu_baseline(R, S, eps, res, target_s):
    """The oracle (plain C, float64) on a bounded sample of rows of the same
    eps-join, on all host cores: its rate, and the element-wise agreement of
    those rows of the timed GPU result with it."""
    import numpy as np

    import oracle
    from paper_1812_07607_amd import synth
    threads = oracle.max_threads()
    n = R.shape[0]
    # grow the sample until one run takes most of target_s (small samples
    # are dominated by thread start-up and load imbalance)
    m = 16
    while True:
        rows = synth.sample_rows(n, m, seed=78)
        t0 = time.perf_counter()
        ref = oracle.eps_join(np.ascontiguousarray(R[rows]), S, eps, row_ids=rows, nthreads=threads,
                              cap=64 * m + 4096)
        dt = time.perf_counter() - t0
        if ref["count"] > 64 * m + 4096:
            ref = oracle.eps_join(np.ascontiguousarray(R[rows]), S, eps, row_ids=rows, nthreads=threads)
        if dt >= 0.6 * target_s or m >= n:
            break
        m = min(n, int(m * min(8.0, max(1.5, 0.9 * target_s / max(dt, 1e-3)))))
    pairs = m * S.shape[0]
    gi, gj, gd = rows_of(res, rows)
    same = bool(len(gi) == ref["count"] and np.array_equal(gi, ref["i"]) and np.array_equal(gj, ref["j"]))
    err = float(np.max(np.abs(gd.astype(np.float64) - ref["dist"]) / np.maximum(ref["dist"], 1e-30))) \
        if same and len(gi) else 0.0
    return {"value": pairs / dt / 1e9, "unit": "G distance-pairs/s", "cores": threads, "cpu": cpu_model(),
            "kind": "oracle",
            "sample": "eps-join of %d seeded rows of R x all %d rows of S (%d pairs, %.1f s); the rate is "
                      "extrapolated from this sample" % (m, S.shape[0], pairs, dt),
            "agreement": {"rows": m, "oracle_pairs": int(ref["count"]), "gpu_pairs": int(len(gi)),
                          "pair_set_identical": same, "max_rel_dist_err": err}}


def serving(args):
    """Resident store of 8,000,000 x 128 unit-norm rows (bf16 operands +
    float32 norms), requests of log-uniform 1..50,000 rows, half eps-join and
    half top-10, Poisson arrivals.  Capacity C is measured closed-loop
    (everything submitted at once); then the offered rate is 0.5 C and 0.8 C
    for a fixed time each; latency is submit -> result ready."""
    import threading

    import numpy as np
    import torch

    from paper_1812_07607_amd import ops, synth
    t0 = time.perf_counter()
    cfg = synth.config5(args.serve_store / 8000000.0)
    S = torch.from_numpy(cfg["S"]).cuda()
    del cfg["S"]
    store = ops.Store(S, "bf16")
    pool = torch.from_numpy(synth.queries_for_store(60000, 128, 1000, seed=505, stream=1)).cuda()
    probe = pool[:256]
    tk = store.join_topk(probe, 10)
    eps = float(torch.median(tk.dist[:, 9]).item())
    t_setup = time.perf_counter() - t0
    srv = ops.Server(store, arena_bytes=48 << 30, n_streams=3, max_batch_requests=64, max_batch_rows=1 << 17)
    arrivals_rng = np.random.default_rng(505)

    def one_run(n_req, rate, seed):
        _, rows, is_topk = synth.request_stream(n_req, max(rate, 1e-6), seed=seed)
        offs = arrivals_rng.integers(0, pool.shape[0] - rows.max(), size=n_req)
        ts = synth.request_stream(n_req, max(rate, 1e-6), seed=seed)[0]
        tickets = []
        done = []
        srv.reset_stats()

        def waiter():
            i = 0
            while i < n_req:
                while i >= len(tickets):
                    time.sleep(0.0005)
                done.append(srv.wait(tickets[i], 120000, fetch=False))
                i += 1

        th = threading.Thread(target=waiter)
        th.start()
        start = time.perf_counter()
        for t in range(n_req):
            if rate > 0:
                delay = ts[t] - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
            q = pool[offs[t]:offs[t] + rows[t]]
            tickets.append(srv.submit(q, "topk" if is_topk[t] else "eps", eps=eps, k=10, sync=False))
        th.join()
        st = srv.stats()
        bad = sum(1 for r in done if r["status"] != 0)
        small = [r["latency_ms"] for r in done if r["rows"] <= 4096 and r["status"] == 0]
        st["small_p50_ms"] = float(np.percentile(small, 50)) if small else None
        st["small_p99_ms"] = float(np.percentile(small, 99)) if small else None
        return st, bad, float(rows.sum())

    def roof(st):
        # matrix-core rate of the served joins (2 d flop per pair) against the
        # dense bf16 peak: over the phase's span, and while batches ran
        flop = 2.0 * 128
        span = st["pairs_done"] * flop / max(st["span_ms"], 1e-9) / 1e9
        per_batch = st["batch_pairs"] * flop / max(st["batch_ms"], 1e-9) / 1e9
        return {"bound": "mfma", "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s", "span_tflops": span,
                "span_frac": span / PEAK_TFLOPS["bf16"], "per_batch_tflops": per_batch,
                "per_batch_frac": per_batch / PEAK_TFLOPS["bf16"],
                "note": "per_batch: summed batch pairs x 2d / summed batch run time (batches overlap on "
                        "the device, so each one's share of the GPU is less than the whole)"}

    torch.cuda.synchronize()
    # closed loop: all requests at once
    progress("serving: store ready (%.1f s); closed-loop capacity run" % t_setup)
    st, bad, rows_c = one_run(64, 0.0, 5051)
    cap_rps = st["completed"] / max(st["span_ms"], 1e-9) * 1e3
    out = {"workload": "resident store %d x 128 bf16; requests log-uniform 1..50,000 rows, 50%% eps (eps=%.4g, "
                       "median 10th-neighbour distance) / 50%% top-10" % (args.serve_store, eps),
           "setup_s": t_setup, "capacity_rps": cap_rps,
           "capacity": {"requests": st["completed"], "gpairs_per_s": st["pairs_done"] / st["span_ms"] * 1e-6,
                        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_batch": st["mean_batch_requests"],
                        "errors": bad, "roofline": roof(st)}}
    for frac in (0.5, 0.8):
        rate = frac * cap_rps
        n_req = max(8, int(rate * args.serve_seconds))
        progress("serving: open loop at %.2f x capacity" % frac)
        st, bad, rows_o = one_run(n_req, rate, 5052 + int(frac * 10))
        out["offered_%.1fC" % frac] = {"rate_rps": rate, "requests": st["completed"],
                                       "gpairs_per_s": st["pairs_done"] / max(st["span_ms"], 1e-9) * 1e-6,
                                       "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "max_ms": st["max_ms"],
                                       "p99_over_p50": st["p99_ms"] / max(st["p50_ms"], 1e-9),
                                       "small_requests_p50_ms": st["small_p50_ms"],
                                       "small_requests_p99_ms": st["small_p99_ms"],
                                       "mean_batch": st["mean_batch_requests"], "errors": bad, "roofline": roof(st)}
    srv.close()
    return out


def per_call(stages, calls, flops):
    """Stage times per call (ms): a call's stage can run several times (the
    bf16 pilot of an E4M3 top-k has its own stages; a capacity retry runs
    the join again), so the sums are divided by the calls made, and the
    number of contractions per call is reported beside them."""
    rec = {k: round(v[0] / calls, 3) for k, v in stages.items() if v[1]}
    rec["contract_tflops"] = round(flops / rec["contract"] / 1e9, 1)
    rec["contractions_per_call"] = round(stages["contract"][1] / calls, 2)
    return rec


def secondary():
    """Stage times of the eps and top-k joins on two unit-vector mixtures
    (200k x 200k at d = 128 with 1,000 centres; 20k queries x 1M rows at
    d = 256 with 4,096 centres), per candidate format: mean of three timed
    calls after one untimed call, stage times from HIP events.  eps is the
    median 10th-neighbour distance of each workload."""
    import torch

    from paper_1812_07607_amd import ops, synth

    torch.cuda.set_device(0)
    ctx = ops.context()
    out = {}

    def run(name, fn, flops):
        try:
            r = fn()
            torch.cuda.synchronize()
        except Exception as e:  # a format that does not converge is reported, not fatal
            out[name] = {"error": str(e)[:160]}
            progress("%s: %s" % (name, out[name]["error"]))
            return
        ctx.timing(reset=True)
        ctx.set_timing(True)
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ctx.set_timing(False)
        st = ctx.timing(reset=True)
        rec = per_call(st, 3, flops)
        if hasattr(r, "candidates"):
            rec.update(candidates=int(r.candidates), pairs=int(r.count))
        else:
            rec.update(band_entries=int(r.band_entries), ties=int(r.ties))
        out[name] = rec
        progress("%s: %s" % (name, json.dumps(rec)))

    def eps_of(R, S):
        # the median 10th-neighbour distance: about ten pairs per query row
        return float(ops.join_topk(R, S, 10, prec="bf16").dist[:, 9].median())

    n = 200000
    R = torch.from_numpy(synth.gaussian_mixture_unit(n, 128, 1000, seed=303)).cuda()
    S = torch.from_numpy(synth.gaussian_mixture_unit(n, 128, 1000, seed=303, stream=1)).cuda()
    fl = 2.0 * n * n * 128
    eps = eps_of(R, S)
    out["eps_200k_d128"] = round(eps, 6)
    for prec in ("bf16", "fp16", "fp8"):
        run("eps_200k_d128_%s" % prec, lambda: ops.join_eps(R, S, eps, prec, max_candidates=1 << 26), fl)
    for prec in ("bf16", "fp16", "fp8"):
        run("top10_200k_d128_%s" % prec, lambda: ops.join_topk(R, S, 10, prec=prec), fl)
    del R, S
    S = torch.from_numpy(synth.gaussian_mixture_unit(1000000, 256, 4096, seed=404)).cuda()
    Q = torch.from_numpy(synth.gaussian_mixture_unit(20000, 256, 4096, seed=404, stream=1)).cuda()
    fl = 2.0 * 20000 * 1000000 * 256
    eps = eps_of(Q, S)
    out["eps_20k_1m_d256"] = round(eps, 6)
    for prec in ("bf16", "fp8"):
        run("eps_20k_1m_d256_%s" % prec, lambda: ops.join_eps(Q, S, eps, prec, max_candidates=1 << 26), fl)
    run("top32_20k_1m_d256_bf16", lambda: ops.join_topk(Q, S, 32, prec="bf16"), fl)
    print(json.dumps({"secondary": out, "data": "synthetic", "timing": "ms per stage per call, mean of 3 calls"}))


def full_configs():
    """The precision-form and FP8-store workloads at full size: a 1M x 1M
    d = 128 mixture (top-10 and eps-join at the median 10th-neighbour
    distance, bf16 candidates against the plain fp32 join) and a 4M x 256
    store probed by 50k queries (top-32, E4M3 and bf16 candidates).  Stage
    times are the mean of two calls after one untimed call."""
    import torch

    from paper_1812_07607_amd import ops, synth

    torch.cuda.set_device(0)
    ctx = ops.context()
    out = {}

    def run(name, fn, flops, reps=2):
        progress("%s ..." % name)
        try:
            r = fn()
            torch.cuda.synchronize()
        except Exception as e:  # reported, not fatal
            out[name] = {"error": str(e)[:200]}
            progress("%s: %s" % (name, out[name]["error"]))
            return None
        ctx.timing(reset=True)
        ctx.set_timing(True)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        ctx.set_timing(False)
        st = ctx.timing(reset=True)
        rec = per_call(st, reps, flops)
        if hasattr(r, "candidates"):
            rec.update(candidates=int(r.candidates), pairs=int(r.count))
        else:
            rec.update(band_entries=int(r.band_entries), ties=int(r.ties))
        out[name] = rec
        progress("%s: %s" % (name, json.dumps(rec)))
        return r

    c3 = synth.config3()
    R = torch.from_numpy(c3["R"]).cuda()
    S = torch.from_numpy(c3["S"]).cuda()
    del c3
    n = R.shape[0]
    fl = 2.0 * n * n * 128
    t = run("c3_top10_bf16", lambda: ops.join_topk(R, S, 10, prec="bf16"), fl)
    eps = float(t.dist[:, 9].median()) if t is not None else 0.6
    out["c3_eps"] = round(eps, 6)
    run("c3_eps_bf16", lambda: ops.join_eps(R, S, eps, "bf16", max_candidates=1 << 26), fl)
    run("c3_eps_fp32", lambda: ops.join_eps(R, S, eps, "fp32", max_candidates=1 << 26), fl, reps=1)
    run("c3_top10_fp32", lambda: ops.join_topk(R, S, 10, prec="fp32"), fl, reps=1)
    del R, S, t
    torch.cuda.empty_cache()
    c4 = synth.config4()
    S = torch.from_numpy(c4["S"]).cuda()
    Q = torch.from_numpy(c4["Q"]).cuda()
    del c4
    fl = 2.0 * Q.shape[0] * S.shape[0] * 256
    run("c4_top32_fp8", lambda: ops.join_topk(Q, S, 32, prec="fp8"), fl)
    run("c4_top32_bf16", lambda: ops.join_topk(Q, S, 32, prec="bf16"), fl)
    print(json.dumps({"full_configs": out, "data": "synthetic",
                      "timing": "ms per stage per call, mean of 2 calls (fp32: 1)"}))


def eps_of_rows(R, S, rows, k=10):
    """eps of the precision-form workload: the lower median, over seeded rows
    of R, of each row's exact k-th neighbour distance in S (the GPU's exact
    top-k)."""
    import numpy as np

    from paper_1812_07607_amd import ops, synth
    import torch
    idx = torch.from_numpy(np.asarray(rows, np.int64)).to(R.device)
    t = ops.join_topk(R.index_select(0, idx).contiguous(), S, k, prec="bf16")
    return float(synth.order_statistic(t.dist[:, k - 1].double().cpu().numpy(), 0.5))


def histogram_leg(args, prec_list, steps):
    """Featurise 100,000 RGB 32x32 patches + the exact eps self-join at the
    0.01% distance quantile, per candidate format: ms per step (featurise
    included), pairs/s, and the pair arrays of every format compared with the
    first one's."""
    import numpy as np
    import torch

    from paper_1812_07607_amd import ops, synth
    ctx = ops.context()
    n = 100000
    cfg = synth.config2(1.0)
    patches = torch.from_numpy(cfg["patches"]).cuda()
    hist = torch.empty((n, 512), dtype=torch.float32, device="cuda")
    ops.featurize_rgb8(patches, 8, out=hist)
    pi, pj = cfg["pairs"]
    d2 = ops.pair_d2(hist, hist, torch.from_numpy(pi), torch.from_numpy(pj)).cpu().numpy()
    eps = float(np.sqrt(synth.order_statistic(d2, cfg["q"])))
    pairs = n * (n - 1) // 2
    out = {"workload": "featurise 100000 RGB 32x32 patches (8x8x8 histograms, 16 base colours + N(0,20^2)) + "
                       "exact eps self-join i<j at the 0.01%% distance quantile (eps %.6g)" % eps}
    first = None
    for prec in prec_list:
        ws = ops.Workspace(hist.device)

        def step():
            ops.featurize_rgb8(patches, 8, out=hist)
            return ops.join_eps(hist, None, eps, prec, workspace=ws)

        r, rec = timed_calls(ctx, step, steps)
        rec["value"] = pairs / (rec["ms_per_call"] * 1e-3) / 1e9
        rec["contract_tflops"] = pairs * 2.0 * 512 / (rec["contract"] * 1e-3) / 1e12
        rec["contract_frac"] = rec["contract_tflops"] / PEAK_TFLOPS[prec]
        rec.update(result_pairs=r.count, candidates=r.candidates, fp64_ties=r.ties)
        if first is None:
            first = r
        else:
            rec["same_pairs_as_" + prec_list[0]] = bool(
                r.count == first.count and torch.equal(r.i, first.i) and torch.equal(r.j, first.j))
        out[prec] = rec
        progress("histogram leg %s: %s" % (prec, json.dumps(rec)))
    return out, {"patches": cfg["patches"], "hist": hist, "eps": eps}


def etl_index_plan_legs():
    """On the 100,000-patch histogram workload: the fused featurise-into-store
    pass and the store self-join against featurise + plain join; the
    index-pruned join against the plain join (fp16 and fp32 candidates); the
    label filter before and after the match; and crop featurisation of boxes
    over frames.  ms per call (mean of 3 after one untimed call), each
    result's pair arrays compared with the plain join's."""
    import numpy as np
    import torch

    from paper_1812_07607_amd import ops, synth
    ctx = ops.context()
    cfg = synth.config2(1.0)
    n = 100000
    pairs = n * (n - 1) // 2
    patches = torch.from_numpy(cfg["patches"]).cuda()
    hist = ops.featurize_rgb8(patches, 8)
    pi, pj = cfg["pairs"]
    d2 = ops.pair_d2(hist, hist, torch.from_numpy(pi), torch.from_numpy(pj)).cpu().numpy()
    eps = float(np.sqrt(synth.order_statistic(d2, cfg["q"])))
    out = {"workload": "100000 palette patches, 8x8x8 histograms, eps self-join at the 0.01%% quantile (eps %.6g)" % eps}

    def same(a, b):
        return bool(a.count == b.count and torch.equal(a.i, b.i) and torch.equal(a.j, b.j))

    # fused featurise-into-store + store self-join vs featurise + join
    plain, rec_p = timed_calls(ctx, lambda: (ops.featurize_rgb8(patches, 8, out=hist),
                                             ops.join_eps(hist, None, eps, "fp16"))[1], 3)
    st_holder = {}
    caps = {}

    def fused():
        st_holder["s"] = ops.Store.featurize(patches, 8, "fp16")
        st_holder["s"]._eps_caps = caps  # the output size that sufficed carries over to the next store
        return st_holder["s"].join_eps_self(eps)

    r, rec_f = timed_calls(ctx, fused, 3)
    out["fused_store"] = {"unfused_ms": rec_p["ms_per_call"], "fused_ms": rec_f["ms_per_call"],
                          "unfused_stages": rec_p, "fused_stages": rec_f, "same_pairs": same(r, plain),
                          "value_fused": pairs / (rec_f["ms_per_call"] * 1e-3) / 1e9}
    progress("fused store: %s" % json.dumps(out["fused_store"]))
    # the index-pruned join
    out["index_join"] = {}
    for prec in ("fp16", "fp32"):
        ref, rec0 = timed_calls(ctx, lambda: ops.join_eps(hist, None, eps, prec), 3)
        (r, info), rec1 = timed_calls(ctx, lambda: ops.join_eps_indexed(hist, None, eps, prec), 3)
        out["index_join"][prec] = {"plain_ms": rec0["ms_per_call"], "indexed_ms": rec1["ms_per_call"],
                                   "speedup": rec0["ms_per_call"] / rec1["ms_per_call"],
                                   "tiles_computed": info.tiles_computed, "tiles_total": info.tiles_total,
                                   "ksteps_computed": info.ksteps_computed,
                                   "ksteps_of_computed_tiles": info.tiles_computed * info.ksteps_per_tile,
                                   "pivots": info.pivots, "indexed_stages": rec1, "same_pairs": same(r, ref),
                                   "value_indexed": pairs / (rec1["ms_per_call"] * 1e-3) / 1e9}
        progress("index %s: %s" % (prec, json.dumps(out["index_join"][prec])))
    # the index-pruned top-10 self-join (each patch's 10 nearest other patches)
    ref, rec0 = timed_calls(ctx, lambda: ops.join_topk(hist, None, 10, exclude_self=True, prec="fp16"), 3)
    (r, info), rec1 = timed_calls(ctx, lambda: ops.join_topk_indexed(hist, None, 10, exclude_self=True,
                                                                     prec="fp16"), 3)
    out["index_top10"] = {"plain_ms": rec0["ms_per_call"], "indexed_ms": rec1["ms_per_call"],
                          "speedup": rec0["ms_per_call"] / rec1["ms_per_call"],
                          "tiles_computed": info.tiles_computed, "tiles_total": info.tiles_total,
                          "ksteps_computed": info.ksteps_computed,
                          "ksteps_of_computed_tiles": info.tiles_computed * info.ksteps_per_tile,
                          "pivots": info.pivots, "plain_stages": rec0, "indexed_stages": rec1,
                          "same_rows": bool(torch.equal(r.j, ref.j) and torch.equal(r.dist, ref.dist))}
    progress("index top-10: %s" % json.dumps(out["index_top10"]))
    del ref, r
    # filter before / after the match (the palette colour as the label)
    labels = torch.from_numpy(cfg["colour"].astype(np.int32)).cuda()
    res = {}
    for plan in ("filter_first", "match_first"):
        res[plan], rec = timed_calls(ctx, lambda: ops.join_eps_filtered(hist, None, eps, labels, None, 5, plan,
                                                                         "fp16"), 3)
        out.setdefault("plans", {})[plan] = {"ms": rec["ms_per_call"], "pairs": res[plan].count}
    out["plans"]["same_pairs"] = same(res["filter_first"], res["match_first"])
    progress("plans: %s" % json.dumps(out["plans"]))
    del hist, patches
    # crops: 20,000 boxes over 64 frames of 720 x 1280
    frames, boxes = synth.frames_with_boxes(64, 720, 1280, 20000, seed=606)
    ft, bt = torch.from_numpy(frames).cuda(), torch.from_numpy(boxes).cuda()
    h2 = torch.empty((boxes.shape[0], 512), dtype=torch.float32, device="cuda")
    _, rec = timed_calls(ctx, lambda: ops.featurize_crops_rgb8(ft, bt, 8, out=h2), 3)
    area = int(((boxes[:, 3] - boxes[:, 1]) * (boxes[:, 4] - boxes[:, 2])).sum())
    nbytes = area * 3 + boxes.shape[0] * 512 * 4
    out["crops"] = {"boxes": int(boxes.shape[0]), "pixels": area, "ms": rec["featurize"],
                    "GBps_algorithmic": nbytes / (rec["featurize"] * 1e-3) / 1e9}
    progress("crops: %s" % json.dumps(out["crops"]))
    return out


def cpu_baseline_crossover():
    """The CPU baseline as a sweep (the CPU-vs-GPU crossover of the paper's
    matching discussion): the histogram self-join at growing sizes, timed as
    the float64 oracle on all host cores against the GPU join on
    device-resident rows and the GPU join with the rows copied in and the
    pairs copied out (an offload from host memory).  The GPU featurises its
    own rows (bit-identical to the oracle's, as the tests check).  One JSON
    line."""
    import numpy as np
    import torch

    import oracle
    from paper_1812_07607_amd import ops, synth
    torch.cuda.set_device(0)
    ctx = ops.context()
    threads = oracle.max_threads()
    cfg = synth.config2(0.4)
    Hfull = oracle.hist_rgb8(cfg["patches"], 8, nthreads=threads)
    Hgpu = ops.featurize_rgb8(torch.from_numpy(cfg["patches"]).cuda(), 8)
    rows = []
    for n in (16, 64, 256, 1024, 4096, 16384, 40000):
        H = np.ascontiguousarray(Hfull[:n])
        Hh = Hgpu[:n].cpu().numpy()  # the GPU's own rows, on the host for the offload timing
        pi, pj = synth.sample_pairs(n, n, 20000, True, seed=n)
        eps = float(np.sqrt(synth.order_statistic(oracle.pair_d2(H, H, pi, pj), 0.001)))
        reps = max(1, min(20, int(2e7 / max(n * n, 1))))
        t0 = time.perf_counter()
        for _ in range(reps):
            ref = oracle.eps_join(H, None, eps, nthreads=threads)
        t_cpu = (time.perf_counter() - t0) / reps
        Hd = Hgpu[:n].contiguous()
        r = ops.join_eps(Hd, None, eps, "fp16")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = ops.join_eps(Hd, None, eps, "fp16")
        torch.cuda.synchronize()
        t_dev = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            Hx = torch.from_numpy(Hh).cuda()
            r = ops.join_eps(Hx, None, eps, "fp16")
            got = (r.i.cpu(), r.j.cpu(), r.dist.cpu())
        t_off = (time.perf_counter() - t0) / reps
        same = bool(r.count == ref["count"] and np.array_equal(got[0].numpy().astype(np.int64), ref["i"]) and
                    np.array_equal(got[1].numpy().astype(np.int64), ref["j"]))
        rows.append({"n": n, "pairs": n * (n - 1) // 2, "cpu_ms": t_cpu * 1e3, "gpu_resident_ms": t_dev * 1e3,
                     "gpu_offload_ms": t_off * 1e3, "same_pairs": same})
        progress("crossover n=%d: %s" % (n, json.dumps(rows[-1])))
    print(json.dumps({"crossover": rows, "cpu": cpu_model(), "cores": threads,
                      "workload": "palette-patch histogram self-join at the 0.1% quantile of 20,000 sampled pairs; "
                                  "GPU fp16 candidates"}))


def store_leg():
    """Top-32 of 50,000 queries against a 4,000,000 x 256 store (4,096-centre
    mixture): E4M3 candidates (with their bf16 pilot) and bf16, ms per call
    (prep of both sides included), the two results compared."""
    import torch

    from paper_1812_07607_amd import ops, synth
    ctx = ops.context()
    c4 = synth.config4()
    S = torch.from_numpy(c4["S"]).cuda()
    Q = torch.from_numpy(c4["Q"]).cuda()
    del c4
    pairs = Q.shape[0] * S.shape[0]
    out = {"workload": "top-32 of 50000 queries x 4000000 x 256 store (4096-centre mixture)"}
    res = {}
    for prec in ("fp8", "bf16"):
        try:
            r, rec = timed_calls(ctx, lambda: ops.join_topk(Q, S, 32, prec=prec), 2)
        except Exception as e:  # reported, not fatal
            out[prec] = {"error": str(e)[:200]}
            continue
        rec["value"] = pairs / (rec["ms_per_call"] * 1e-3) / 1e9
        rec.update(band_entries=r.band_entries, ties=r.ties)
        res[prec] = r
        out[prec] = rec
        progress("store leg %s: %s" % (prec, json.dumps(rec)))
    if len(res) == 2:
        out["same_neighbours"] = bool(torch.equal(res["fp8"].j, res["bf16"].j))
        if "ms_per_call" in out.get("fp8", {}):
            out["fp8_speedup_end_to_end"] = out["bf16"]["ms_per_call"] / out["fp8"]["ms_per_call"]
    return out


def histogram_headline(args):
    """The featurise + self-join step alone (profiling runs of that kernel)."""
    import numpy as np
    prec = args.prec if args.prec != "bf16" else "fp16"
    leg, _ = histogram_leg(args, [prec], args.steps)
    rec = leg[prec]
    pairs = 100000 * 99999 // 2
    res = {"metric": METRIC, "value": rec["value"], "unit": "G distance-pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": rec["ms_per_call"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
           "config": {"workload": leg["workload"], "pairs": pairs},
           "roofline": {"kernel": "cand_kernel<%s, eps>" % prec, "bound": "mfma", "achieved": rec["contract_tflops"],
                        "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s", "frac": rec["contract_frac"],
                        "traffic": measured_traffic(prec, "featurise + eps self-join, 100000 patches"),
                        "flops_per_launch": pairs * 2.0 * 512, "avg_launch_ms": rec["contract"]}}
    del np
    print(json.dumps(res))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.secondary:
        secondary()
        return
    if args.full_configs:
        full_configs()
        return
    import numpy as np
    import torch

    from paper_1812_07607_amd import ops, synth

    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.histogram_headline:
        histogram_headline(args)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving(args)}))
        return
    if args.etl_only:
        print(json.dumps({"etl_index_plans": etl_index_plan_legs()}))
        return
    if args.crossover:
        cpu_baseline_crossover()
        return
    n = args.n
    d = 128
    c3 = synth.config3(n / 1000000.0)
    R_h, S_h = c3["R"], c3["S"]
    del c3
    R = torch.from_numpy(R_h).cuda()
    S = torch.from_numpy(S_h).cuda()
    n = R.shape[0]
    eps = eps_of_rows(R, S, synth.sample_rows(n, 256, seed=3031))
    ctx = ops.context()
    ws = ops.Workspace(R.device)

    def step(prec, out=None):
        return ops.join_eps(R, S, eps, prec, workspace=ws, out=out, max_candidates=1 << 26)

    progress("setup done (eps %.6g); warm-up and %d timed steps" % (eps, args.steps))
    r = step(args.prec)
    cap = max(r.count + r.count // 4, 1 << 16)
    out = (torch.empty(cap, dtype=torch.int32, device="cuda"), torch.empty(cap, dtype=torch.int32, device="cuda"),
           torch.empty(cap, dtype=torch.float32, device="cuda"))
    for _ in range(args.warmup):
        step(args.prec, out)
    torch.cuda.synchronize()
    ctx.timing(reset=True)
    ctx.set_timing(True)
    lat = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        r = step(args.prec, out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    ctx.set_timing(False)
    stages = ctx.timing(reset=True)
    pairs = n * n
    ms_step = elapsed / args.steps * 1e3
    value = pairs / (elapsed / args.steps) / 1e9
    progress("timed steps: %.3f ms/step" % ms_step)

    # dominant kernel: the matrix-core contraction (stage "contract")
    c_ms, c_calls = stages["contract"]
    c_avg = c_ms / max(c_calls, 1)
    flops = pairs * 2.0 * d
    achieved = flops / (c_avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.prec]
    workload = "eps-join %d x %d, d=128, unit-norm 1000-centre mixture" % (n, n)
    roof = {"kernel": "cand_kernel<%s, eps>" % args.prec, "bound": "mfma", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": measured_traffic(args.prec, workload),
            "flops_per_launch": flops, "avg_launch_ms": c_avg}
    # the achievable rates of this device (register-operand matrix-core loop,
    # 1 GiB copy), measured once after the timed steps: the second denominator
    progress("measured peaks")
    peaks = ops.measure_peaks()
    roof["measured_peak"] = peaks[args.prec]
    roof["frac_of_measured_peak"] = achieved / peaks[args.prec]
    res = {
        "metric": METRIC, "value": value, "unit": "G distance-pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "exact eps-join of R = S-size %d x 128 unit-norm float32 vectors (1,000-centre "
                               "Gaussian mixture, sigma 0.05; R and S independent draws) at eps = lower median "
                               "exact 10th-neighbour distance of 256 seeded rows; %s candidates, float32/float64 "
                               "recheck, (i, j)-ordered output" % (n, args.prec),
                   "rows_R": n, "rows_S": n, "dim": d, "pairs": pairs, "eps": eps, "result_pairs": r.count,
                   "candidates": r.candidates, "fp64_ties": r.ties},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "stages_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in stages.items() if v[1]},
        "roofline": roof,
        "measured_peaks": {"mfma_tflops": {k: peaks[k] for k in ("fp32", "bf16", "fp16", "fp8")},
                           "mfma_bf16_tflops_at_2_waves_per_simd": {
                               "16x16x32": peaks["bf16_16x16x32_2_waves_per_simd"],
                               "32x32x16": peaks["bf16_32x32x16_2_waves_per_simd"],
                               "16x16x32_lds_fed_candidate_loop": peaks["bf16_lds_fed_candidate_loop"]},
                           "hbm_copy_GBps": peaks["hbm_copy_GBps"], "hbm_read_GBps": peaks["hbm_read_GBps"],
                           "how": "dl_measure_peaks: 8 independent MFMA chains per wave, 32 waves per CU, register "
                                  "operands (and 8 waves per CU, the candidate pass's occupancy, with register "
                                  "operands or with the pass's LDS fragment reads and a barrier per K-step); a 1 GiB device "
                                  "copy (bytes read + written) and a 1 GiB streaming read"},
    }
    if not args.no_extras:
        if args.prec != "fp32":
            # the plain fp32 GPU join on the same input: time and pair arrays
            progress("plain fp32 join")
            r32, rec = timed_calls(ctx, lambda: step("fp32"), 1)
            rec["value"] = pairs / (rec["ms_per_call"] * 1e-3) / 1e9
            rec["contract_tflops"] = flops / (rec["contract"] * 1e-3) / 1e12
            rec["same_pairs"] = bool(r32.count == r.count and torch.equal(r32.i, r.i[:r.count])
                                     and torch.equal(r32.j, r.j[:r.count]))
            rec["speedup_of_%s" % args.prec] = rec["ms_per_call"] / ms_step
            res["fp32_join"] = rec
            del r32
        progress("top-10 join")
        t, rec = timed_calls(ctx, lambda: ops.join_topk(R, S, 10, prec=args.prec, workspace=ws), 2)
        rec["value"] = pairs / (rec["ms_per_call"] * 1e-3) / 1e9
        rec["contract_tflops"] = flops / (rec["contract"] * 1e-3) / 1e12
        rec.update(band_entries=t.band_entries, ties=t.ties)
        res["top10_join"] = rec
        del t
        torch.cuda.empty_cache()
    # the oracle leg needs the timed result; keep its rows on the host
    gpu_res = r
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle, about %.0f s)" % args.cpu_seconds)
        res["cpu_baseline"] = cpu_baseline(R_h, S_h, eps, gpu_res, args.cpu_seconds)
    del R, S, ws, out, gpu_res, r
    torch.cuda.empty_cache()
    if not args.no_extras:
        progress("histogram leg")
        res["histogram_join"], _ = histogram_leg(args, ["fp32", "fp16"], 3)
        torch.cuda.empty_cache()
        progress("fused store, index, plan and crop legs")
        res["etl_index_plans"] = etl_index_plan_legs()
        torch.cuda.empty_cache()
        progress("store leg")
        res["store_top32"] = store_leg()
        torch.cuda.empty_cache()
        if not args.no_serving:
            try:
                res["serving"] = serving(args)
            except Exception as e:  # reported, not fatal to the main measurement
                res["serving"] = {"error": repr(e)}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
