"""Benchmark: featurise + exact eps self-join of 100,000 RGB patches on one GPU.

One step is the whole hot path over one batch of synthetic input already
resident in HBM: colour histograms of 100,000 uint8 32x32 patches (8x8x8
bins), operand prep, the matrix-core candidate pass with the fused eps
filter, the float32 / float64 recheck and the canonical (i, j) sort, for the
self-join i < j at the 0.01% distance quantile.  `value` is the number of
distance pairs in the join's domain (n(n-1)/2) per second of step time.

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
    ap.add_argument("--prec", default="fp16", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--n", type=int, default=100000, help="patches (default: the full workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--no-fp32-compare", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-store", type=int, default=8000000, help="rows of the serving store")
    ap.add_argument("--serve-seconds", type=float, default=6.0, help="open-loop seconds per offered rate")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="copy this many MiB device-to-device first (scale for FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--secondary", action="store_true",
                    help="instead of the headline step, time the unit-mixture eps and top-k joins (one JSON line)")
    ap.add_argument("--full-configs", action="store_true",
                    help="instead of the headline step, time the 1M x 1M d=128 joins (bf16 and fp32) and the "
                         "4M x 256 store with 50k top-32 queries (fp8 and bf16) at full size (one JSON line)")
    return ap.parse_args()


KERNEL_SOURCES = ["paper_1812_07607_amd/csrc/join_mfma.hip", "paper_1812_07607_amd/csrc/join_params.hpp",
                  "paper_1812_07607_amd/csrc/dl_internal.hpp"]
TRAFFIC_SUMMARY = "profiles/cand_kernel_fp16_selfjoin_100k_traffic.txt"


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


def measured_traffic(prec):
    """HBM bytes per launch of the contraction kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source
    (else None)."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if prec != "fp16" or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(H, eps, n, target_s):
    """The oracle (plain C, float64) on a bounded sample of rows of the same
    self-join, on all host cores."""
    import numpy as np

    import oracle
    from paper_1812_07607_amd import synth
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    feat = oracle.hist_rgb8(H["patches"][:2000], 8, nthreads=threads)
    t_feat = (time.perf_counter() - t0) / 2000
    del feat
    Hn = H["hist"]
    # grow the sample until one run takes most of target_s (small samples
    # are dominated by thread start-up and load imbalance)
    m = 16
    while True:
        rows = synth.sample_rows(n, m, seed=78)
        pairs = int(sum(n - 1 - r for r in rows))
        t0 = time.perf_counter()
        oracle.eps_join(np.ascontiguousarray(Hn[rows]), Hn, eps, self_join=True, row_ids=rows, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * target_s or m >= n:
            break
        m = min(n, int(m * min(8.0, max(1.5, 0.9 * target_s / max(dt, 1e-3)))))
    return {"value": pairs / dt / 1e9, "unit": "G distance-pairs/s", "cores": threads, "kind": "oracle",
            "sample": "eps self-join of %d seeded rows x all later rows (%d pairs, %.1f s); featurise %.2f us/patch "
                      "(not in value)" % (m, pairs, dt, t_feat * 1e6)}


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
        return st, bad, float(rows.sum())

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
                        "errors": bad}}
    for frac in (0.5, 0.8):
        rate = frac * cap_rps
        n_req = max(8, int(rate * args.serve_seconds))
        progress("serving: open loop at %.2f x capacity" % frac)
        st, bad, rows_o = one_run(n_req, rate, 5052 + int(frac * 10))
        out["offered_%.1fC" % frac] = {"rate_rps": rate, "requests": st["completed"],
                                       "gpairs_per_s": st["pairs_done"] / max(st["span_ms"], 1e-9) * 1e-6,
                                       "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "max_ms": st["max_ms"],
                                       "mean_batch": st["mean_batch_requests"], "errors": bad}
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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
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
    n = args.n
    cfg = synth.config2(n / 100000.0)
    patches = torch.from_numpy(cfg["patches"]).cuda()
    hist = torch.empty((n, 512), dtype=torch.float32, device="cuda")
    ops.featurize_rgb8(patches, 8, out=hist)
    pi, pj = cfg["pairs"]
    d2 = ops.pair_d2(hist, hist, torch.from_numpy(pi), torch.from_numpy(pj)).cpu().numpy()
    eps = float(np.sqrt(synth.order_statistic(d2, cfg["q"])))
    ctx = ops.context()
    ws = ops.Workspace(hist.device)

    def step(prec, out=None):
        ops.featurize_rgb8(patches, 8, out=hist)
        return ops.join_eps(hist, None, eps, prec, workspace=ws, out=out)

    progress("setup done (eps %.6g); warm-up and %d timed steps" % (eps, args.steps))
    r = step(args.prec)
    cap = max(r.count * 2, 1 << 16)
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
    pairs = n * (n - 1) // 2
    ms_step = elapsed / args.steps * 1e3
    value = pairs / (elapsed / args.steps) / 1e9

    # dominant kernel: the matrix-core contraction (stage "contract")
    c_ms, c_calls = stages["contract"]
    c_avg = c_ms / max(c_calls, 1)
    flops = pairs * 2.0 * 512
    achieved = flops / (c_avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.prec]
    roof = {"kernel": "cand_kernel<%s, eps>" % args.prec, "bound": "mfma", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": measured_traffic(args.prec),
            "flops_per_launch": flops, "avg_launch_ms": c_avg}
    res = {
        "metric": METRIC, "value": value, "unit": "G distance-pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "featurise %d RGB 32x32 patches (8x8x8 histograms, 16 base colours + N(0,20^2)) + "
                               "exact eps self-join i<j at the 0.01%% distance quantile" % n,
                   "patches": n, "dim": 512, "pairs": pairs, "eps": eps, "result_pairs": r.count,
                   "candidates": r.candidates, "fp64_ties": r.ties},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "stages_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in stages.items() if v[1]},
        "roofline": roof,
    }
    progress("timed steps: %.3f ms/step" % ms_step)
    if not args.no_fp32_compare and args.prec != "fp32":
        # the plain fp32 GPU join on the same input, for comparison
        step("fp32", out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k32 = max(1, min(3, args.steps))
        for _ in range(k32):
            r32 = step("fp32", out)
        torch.cuda.synchronize()
        t32 = (time.perf_counter() - t0) / k32
        res["fp32_join"] = {"value": pairs / t32 / 1e9, "ms_per_step": t32 * 1e3, "candidates": r32.candidates,
                            "same_pairs": bool(r32.count == r.count)}
    if not args.no_serving:
        try:
            res["serving"] = serving(args)
        except Exception as e:  # reported, not fatal to the main measurement
            res["serving"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle, about %.0f s)" % args.cpu_seconds)
        res["cpu_baseline"] = cpu_baseline({"patches": cfg["patches"], "hist": hist.cpu().numpy()}, eps, n,
                                           args.cpu_seconds)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
