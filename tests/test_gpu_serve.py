"""Resident store and serving loop on the GPU.

Store joins equal the oracle; every served request's result equals (bit for
bit) the same request run alone through the store call, whatever batch it
was packed into; memory admission, rejection and cancellation behave as
documented."""
import numpy as np
import pytest
import torch

from gpu_util import assert_eps_equal, assert_topk_equal, dev, host
from paper_1812_07607_amd import ops, synth
from paper_1812_07607_amd._lib import DL_ERR_CANCELLED, DL_ERR_OOM, DL_OK, DLError

pytestmark = pytest.mark.gpu

D = 64
WAIT_MS = 60000  # a request not done within a minute fails the test instead of stalling it


@pytest.fixture(scope="module")
def store_data():
    S = synth.gaussian_mixture_unit(30000, D, 200, seed=505)
    return S


@pytest.mark.parametrize("prec", ["bf16", "fp8", "fp32"])
def test_store_joins_match_oracle(orc, store_data, prec):
    S = store_data
    st = ops.Store(dev(S), prec)
    Q = synth.gaussian_mixture_unit(300, D, 200, seed=505, stream=7)
    ref_j, ref_d2, ref_dist = orc.topk(Q, S, 10)
    got = st.join_topk(dev(Q), 10)
    assert_topk_equal(got, ref_j, ref_dist, D, "store top-10/" + prec)
    eps = float(np.median(np.sqrt(ref_d2[:, 9])))
    ref = orc.eps_join(Q, S, eps)
    got = st.join_eps(dev(Q), eps)
    assert_eps_equal(got, ref, D, "store eps/" + prec)


def _requests(n, seed, max_rows=400):
    rng = np.random.default_rng(seed)
    rows = np.clip(np.rint(np.exp(rng.uniform(0, np.log(max_rows), size=n))), 1, max_rows).astype(int)
    modes = np.where(rng.random(n) < 0.5, "eps", "topk")
    qs = [synth.gaussian_mixture_unit(int(r), D, 200, seed=505, stream=100 + t) for t, r in enumerate(rows)]
    return qs, modes


def _same(a, b):
    return all(torch.equal(a[k], b[k]) for k in ("j", "dist")) and ("i" not in a or torch.equal(a["i"], b["i"]))


def test_results_alone_equal_results_in_mix(orc, store_data):
    S = store_data
    st = ops.Store(dev(S), "bf16")
    # eps: the median 10th-neighbour distance of a seeded query sample
    probe = synth.gaussian_mixture_unit(256, D, 200, seed=505, stream=99)
    _, d2, _ = orc.topk(probe, S, 10)
    eps = float(np.median(np.sqrt(d2[:, 9])))
    qs, modes = _requests(40, seed=3)
    srv = ops.Server(st, arena_bytes=1 << 30, n_streams=2, max_batch_requests=16)
    try:
        # alone: one request at a time on an idle server
        alone = []
        for q, m in zip(qs, modes):
            t = srv.submit(dev(q), m, eps=eps, k=10)
            alone.append(srv.wait(t, WAIT_MS))
        assert all(r["batch_requests"] == 1 for r in alone)
        # mix: everything at once
        tq = [dev(q) for q in qs]
        tickets = [srv.submit(q, m, eps=eps, k=10) for q, m in zip(tq, modes)]
        mixed = [srv.wait(t, WAIT_MS) for t in tickets]
        assert max(r["batch_requests"] for r in mixed) > 1, "nothing was batched"
        for a, b, m in zip(alone, mixed, modes):
            assert a["status"] == DL_OK and b["status"] == DL_OK
            assert _same(a, b), "result changed when batched (%s)" % m
        # and both equal the oracle on a sample of requests
        for t in range(0, 40, 5):
            q, m, r = qs[t], modes[t], mixed[t]
            if m == "topk":
                ref_j, _, ref_dist = orc.topk(q, S, 10)
                assert_topk_equal(ops.TopkResult(r["j"].view(torch.int32), r["dist"], 0, 0), ref_j, ref_dist, D,
                                  "served top-k %d" % t)
            else:
                ref = orc.eps_join(q, S, eps)
                res = ops.EpsResult(r["i"].view(torch.int32), r["j"].view(torch.int32), r["dist"], r["count"], 0, 0)
                assert_eps_equal(res, ref, D, "served eps %d" % t)
        s = srv.stats()
        assert s["completed"] == 80 and s["rejected"] == 0 and s["p99_ms"] >= s["p50_ms"] > 0
    finally:
        srv.close()


def test_memory_admission_and_rejection(orc, store_data):
    S = store_data
    st = ops.Store(dev(S), "bf16")
    qs, modes = _requests(24, seed=4, max_rows=64)
    # an arena that holds only a few small batches at a time
    srv = ops.Server(st, arena_bytes=48 << 20, n_streams=3, max_batch_requests=4)
    try:
        tickets = [srv.submit(dev(q), m, eps=0.3, k=10) for q, m in zip(qs, modes)]
        res = [srv.wait(t, WAIT_MS) for t in tickets]
        assert all(r["status"] == DL_OK for r in res)
        s = srv.stats()
        assert s["arena_peak"] <= 48 << 20
        # a request that cannot fit an empty arena is rejected, not hung
        big = dev(synth.gaussian_mixture_unit(60000, D, 200, seed=505, stream=5))
        t = srv.submit(big, "topk", k=10)
        assert srv.wait(t, WAIT_MS)["status"] == DL_ERR_OOM
        # the server still works afterwards
        t = srv.submit(dev(qs[0]), modes[0], eps=0.3, k=10)
        assert srv.wait(t, WAIT_MS)["status"] == DL_OK
    finally:
        srv.close()


def test_cancel_and_invalid(store_data):
    st = ops.Store(dev(store_data), "bf16")
    srv = ops.Server(st, arena_bytes=1 << 30, n_streams=1, max_batch_requests=1)
    try:
        qs = [dev(synth.gaussian_mixture_unit(2000, D, 200, seed=505, stream=200 + t)) for t in range(6)]
        tickets = [srv.submit(q, "topk", k=10) for q in qs]
        cancelled = srv.cancel(tickets[-1])
        res = [srv.wait(t, WAIT_MS) for t in tickets]
        if cancelled:
            assert res[-1]["status"] == DL_ERR_CANCELLED
        assert all(r["status"] == DL_OK for r in res[:-1])
        with pytest.raises(DLError):
            srv.submit(dev(np.zeros((3, D + 1), np.float32)), "eps", eps=0.1)
        with pytest.raises(DLError):
            srv.submit(dev(np.zeros((3, D), np.float32)), "topk", k=0)
        t = srv.submit(dev(np.zeros((0, D), np.float32)), "eps", eps=0.1)
        assert srv.wait(t, WAIT_MS)["status"] == DL_OK
    finally:
        srv.close()


def test_batch_capacity_overflow_does_not_fail_batch_mates(orc, store_data):
    """Requests whose pairs fit the per-batch output capacity alone but not
    together (and one that does not fit it even alone): every request still
    succeeds, with the result it has alone, equal to the oracle's."""
    S = store_data
    st = ops.Store(dev(S), "bf16")
    probe = synth.gaussian_mixture_unit(64, D, 200, seed=505, stream=98)
    pi, pj = np.meshgrid(np.arange(64), np.arange(S.shape[0]), indexing="ij")
    d2 = orc.pair_d2(probe, S, pi.ravel(), pj.ravel())
    # about 20,000 store rows per query row: four rows overflow 65,536 pairs
    eps = float(np.sqrt(np.sort(d2)[int(len(d2) * 20000 / S.shape[0])]))
    qs = [synth.gaussian_mixture_unit(n, D, 200, seed=505, stream=300 + t) for t, n in enumerate([1, 1, 1, 1, 1, 5, 2])]
    srv = ops.Server(st, arena_bytes=2 << 30, n_streams=1, max_batch_requests=16, pairs_per_row=64)
    try:
        tq = [dev(q) for q in qs]
        # one worker: the first request runs while the rest queue up and are batched
        tickets = [srv.submit(q, "eps", eps=eps) for q in tq]
        mixed = [srv.wait(t, WAIT_MS) for t in tickets]
        alone = []
        for q in tq:
            t = srv.submit(q, "eps", eps=eps)
            alone.append(srv.wait(t, WAIT_MS))
    finally:
        srv.close()
    for t, (a, b) in enumerate(zip(alone, mixed)):
        assert a["status"] == DL_OK and b["status"] == DL_OK, "request %d: %d alone, %d in the mix" % (
            t, a["status"], b["status"])
        assert _same(a, b), "request %d changed when batched" % t
        ref = orc.eps_join(qs[t], S, eps)
        res = ops.EpsResult(b["i"].view(torch.int32), b["j"].view(torch.int32), b["dist"], b["count"], 0, 0)
        assert_eps_equal(res, ref, D, "overflowing eps request %d" % t)
    assert sum(r["count"] for r in mixed) > 65536
    assert max(r["count"] for r in mixed) > 65536  # the 5-row request alone outgrows the default
