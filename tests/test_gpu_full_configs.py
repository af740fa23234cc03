"""GPU parity at the full sizes of the three large workloads, against the
float64 oracle on seeded rows (rows of a join are independent, so a sample
of rows is checked exactly at any size):

* 1,000,000 x 1,000,000 unit vectors, d = 128: the bf16 eps-join at the
  lower median exact 10th-neighbour distance, and the bf16 top-10;
* a 4,000,000 x 256 store probed by 50,000 queries: E4M3 top-32;
* an 8,000,000 x 128 bf16 store behind the serving loop: requests of
  log-uniform size (1..50,000 rows), half eps-join and half top-10, every
  result bit-identical alone and in the mix.
The GPU runs each join whole, in the same call shape the benchmark times."""
import numpy as np
import pytest
import torch

from gpu_util import assert_dist_close, assert_topk_equal, dev, host
from paper_1812_07607_amd import ops, synth
from paper_1812_07607_amd._lib import DL_OK

pytestmark = pytest.mark.gpu


def eps_pairs_of_rows(res, rows):
    gi = res.i.long() & 0xffffffff
    keep = torch.isin(gi, dev(np.asarray(rows, np.int64)))
    return host(gi[keep]), host(res.j.long()[keep] & 0xffffffff), host(res.dist[keep])


def check_eps_rows(orc, res, R, S, eps, rows, d, what):
    gi, gj, gd = eps_pairs_of_rows(res, rows)
    ref = orc.eps_join(np.ascontiguousarray(R[rows]), S, eps, row_ids=rows, cap=max(4096, 256 * len(rows)))
    assert ref["count"] <= max(4096, 256 * len(rows))
    missing = len(set(zip(ref["i"].tolist(), ref["j"].tolist())) - set(zip(gi.tolist(), gj.tolist())))
    assert missing == 0, "%s: %d oracle pairs missing from the GPU result" % (what, missing)
    assert len(gi) == ref["count"], "%s: %d pairs vs oracle %d" % (what, len(gi), ref["count"])
    assert np.array_equal(gi, ref["i"]) and np.array_equal(gj, ref["j"]), what + ": (i, j) differ"
    assert_dist_close(gd, ref["dist"], d, what)
    return ref["count"]


def eps_from_probe(orc, R, S, nprobe, seed):
    """Lower median, over seeded rows, of the exact 10th-neighbour distance."""
    rows = synth.sample_rows(R.shape[0], nprobe, seed=seed)
    _, _, dist = orc.topk(np.ascontiguousarray(R[rows]), S, 10)
    return float(synth.order_statistic(dist[:, 9].astype(np.float64), 0.5))


@pytest.fixture(scope="module")
def c3():
    cfg = synth.config3()
    return cfg["R"], cfg["S"]


def test_precision_form_eps_join_full_size(orc, c3):
    R, S = c3
    eps = eps_from_probe(orc, R, S, 256, 3031)
    res = ops.join_eps(dev(R), dev(S), eps, "bf16", max_candidates=1 << 26)
    assert res.count > 10 * R.shape[0] // 2
    # (i, j) order over the whole result
    key = (res.i.long() & 0xffffffff) * (1 << 32) + (res.j.long() & 0xffffffff)
    assert bool((key[1:] > key[:-1]).all())
    rows = synth.sample_rows(R.shape[0], 2000, seed=3032)
    m = check_eps_rows(orc, res, R, S, eps, rows, 128, "1M x 1M bf16 eps, 2,000 seeded rows")
    assert m > 2000


def test_precision_form_top10_full_size(orc, c3):
    R, S = c3
    got = ops.join_topk(dev(R), dev(S), 10, prec="bf16")
    rows = synth.sample_rows(R.shape[0], 2000, seed=3033)
    ref_j, _, ref_dist = orc.topk(np.ascontiguousarray(R[rows]), S, 10)
    idx = dev(rows).long()
    assert_topk_equal(ops.TopkResult(got.j[idx], got.dist[idx], 0, 0), ref_j, ref_dist, 128,
                      "1M x 1M bf16 top-10, 2,000 seeded rows")


def test_fp8_store_top32_full_size(orc):
    cfg = synth.config4()
    S, Q = cfg["S"], cfg["Q"]
    del cfg
    St, Qt = dev(S), dev(Q)
    got = ops.join_topk(Qt, St, 32, prec="fp8")
    rows = synth.sample_rows(Q.shape[0], 500, seed=4041)
    ref_j, _, ref_dist = orc.topk(np.ascontiguousarray(Q[rows]), S, 32)
    idx = dev(rows).long()
    assert_topk_equal(ops.TopkResult(got.j[idx], got.dist[idx], 0, 0), ref_j, ref_dist, 256,
                      "4M x 256 store, 50,000 queries, E4M3 top-32, 500 seeded rows")
    # the whole neighbour list equals the bf16 pass's (both are exact)
    ref16 = ops.join_topk(Qt, St, 32, prec="bf16")
    assert torch.equal(got.j, ref16.j)


def test_serving_full_store(orc):
    cfg = synth.config5()
    S = cfg["S"]
    del cfg
    St = dev(S)
    store = ops.Store(St, "bf16")
    pool = synth.queries_for_store(60000, 128, 1000, seed=505, stream=1)
    eps = eps_from_probe(orc, pool, S, 64, 5051)
    _, sizes, is_topk = synth.request_stream(16, 1.0, seed=5053)
    offs = np.random.default_rng(5054).integers(0, pool.shape[0] - sizes.max(), size=16)
    qs = [pool[o:o + n] for o, n in zip(offs, sizes)]
    modes = ["topk" if t else "eps" for t in is_topk]
    srv = ops.Server(store, arena_bytes=16 << 30, n_streams=3, max_batch_requests=16, max_batch_rows=1 << 17)
    try:
        alone = []
        for q, m in zip(qs, modes):
            t = srv.submit(dev(q), m, eps=eps, k=10)
            alone.append(srv.wait(t, 120000))
        tq = [dev(q) for q in qs]
        tickets = [srv.submit(q, m, eps=eps, k=10) for q, m in zip(tq, modes)]
        mixed = [srv.wait(t, 120000) for t in tickets]
    finally:
        srv.close()
    assert max(r["batch_requests"] for r in mixed) > 1, "nothing was batched"
    for t, (a, b, m) in enumerate(zip(alone, mixed, modes)):
        assert a["status"] == DL_OK and b["status"] == DL_OK, "request %d: %s / %s" % (t, a["status"], b["status"])
        for key in ("j", "dist") + (("i",) if m == "eps" else ()):
            assert torch.equal(a[key], b[key]), "request %d (%s): %s changed when batched" % (t, m, key)
    # each request against the oracle on up to 8 seeded rows
    for t, (q, m, r) in enumerate(zip(qs, modes, mixed)):
        rows = synth.sample_rows(q.shape[0], 8, seed=5060 + t)
        if m == "topk":
            ref_j, _, ref_dist = orc.topk(np.ascontiguousarray(q[rows]), S, 10)
            idx = dev(rows).long()
            assert_topk_equal(ops.TopkResult(r["j"].view(torch.int32)[idx], r["dist"][idx], 0, 0), ref_j, ref_dist,
                              128, "served top-10, request %d" % t)
        else:
            res = ops.EpsResult(r["i"].view(torch.int32), r["j"].view(torch.int32), r["dist"], r["count"], 0, 0)
            check_eps_rows(orc, res, q, S, eps, rows, 128, "served eps, request %d" % t)
