"""A seeded sweep of small joins against the oracle, all four candidate
formats: random shapes (ragged against the 256-row tiles and the 64- and
128-byte K-steps), self-joins and two-relation joins, four value
distributions (unit-norm mixture, uniform, integer grid with ties, scaled
magnitudes with planted duplicates), eps either at a sampled pair-distance
quantile or exactly at a pair's distance (the inclusive boundary), and
top-k with k from 1 to past the relation's size.  Pairs and indices must
equal the oracle's exactly; distances within the float32 bound."""
import numpy as np
import pytest

from gpu_util import assert_eps_equal, assert_topk_equal, dev
from paper_1812_07607_amd import ops, synth

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "bf16", "fp16", "fp8"]
CASES = 32


def draw_case(seed):
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(1, 900))
    self_join = bool(rng.random() < 0.3)
    m = n if self_join else int(rng.integers(1, 1100))
    d = int(rng.choice([1, 3, 17, 64, 127, 128, 129, 200, 300]))
    kind = int(rng.integers(0, 4))
    if kind == 0:
        R = synth.gaussian_mixture_unit(n, d, max(1, n // 40), seed=seed)
        S = synth.gaussian_mixture_unit(m, d, max(1, n // 40), seed=seed, stream=1)
    elif kind == 1:
        R = synth.uniform_rows(n, d, seed=seed)
        S = synth.uniform_rows(m, d, seed=seed, stream=1)
    elif kind == 2:
        R = synth.integer_grid_rows(n, d, levels=3, seed=seed)
        S = synth.integer_grid_rows(m, d, levels=3, seed=seed, stream=1)
    else:
        scale = float(10.0 ** rng.integers(-12, 12))
        R = (synth.uniform_rows(n, d, seed=seed) * scale).astype(np.float32)
        S = (synth.uniform_rows(m, d, seed=seed, stream=1) * scale).astype(np.float32)
        S[rng.integers(0, m, size=max(1, m // 10))] = R[rng.integers(0, n, size=max(1, m // 10))]
    if self_join:
        S = R
    return rng, R, S, self_join, d


@pytest.mark.parametrize("prec", PRECS)
def test_random_eps_joins(orc, prec):
    for seed in range(CASES):
        rng, R, S, self_join, d = draw_case(seed)
        n, m = len(R), len(S)
        if self_join and n < 2:
            continue
        pi, pj = synth.sample_pairs(n, m, 4000, self_join, seed=seed)
        d2 = orc.pair_d2(R, S, pi, pj)
        if rng.random() < 0.5:
            eps = float(np.sqrt(synth.order_statistic(d2, float(rng.choice([0.001, 0.01, 0.05])))))
        else:
            eps = float(np.sqrt(d2[int(rng.integers(0, len(d2)))]))  # a pair exactly on the boundary
        ref = orc.eps_join(R, None if self_join else S, eps)
        got = ops.join_eps(dev(R), None if self_join else dev(S), eps, prec)
        assert_eps_equal(got, ref, d, "seed %d n %d m %d d %d self %s eps %.9g/%s" % (
            seed, n, m, d, self_join, eps, prec))


@pytest.mark.parametrize("prec", PRECS)
def test_random_topk_joins(orc, prec):
    for seed in range(CASES):
        rng, R, S, self_join, d = draw_case(seed)
        m = len(S)
        k = int(rng.integers(1, min(40, m + 3) + 1))
        excl = self_join and bool(rng.random() < 0.5)
        ref_j, _, ref_dist = orc.topk(R, None if self_join else S, k, exclude_self=excl)
        got = ops.join_topk(dev(R), None if self_join else dev(S), k, exclude_self=excl, prec=prec)
        assert_topk_equal(got, ref_j, ref_dist, d, "seed %d n %d m %d d %d k %d self %s excl %s/%s" % (
            seed, len(R), m, d, k, self_join, excl, prec))


def draw_clustered(seed):
    """Relations of 257..4,000 rows (at least two tiles each, so the index
    is built) with cluster structure the index can prune on: a tight
    mixture of a few centres, Dirichlet histograms, or rows nonzero in one
    of eight coordinate blocks (whose zero K-steps are skipped)."""
    rng = np.random.default_rng(9500 + seed)
    n = int(rng.integers(257, 4000))
    self_join = bool(rng.random() < 0.5)
    m = n if self_join else int(rng.integers(257, 4000))
    kind = int(rng.integers(0, 3))
    if kind == 0:
        d = int(rng.choice([32, 64, 128]))
        c = int(rng.integers(4, 13))
        R = synth.gaussian_mixture_unit(n, d, c, sigma=0.02, seed=seed)
        S = synth.gaussian_mixture_unit(m, d, c, sigma=0.02, seed=seed, stream=1)
    elif kind == 1:
        d = 64
        R = synth.dirichlet_clusters(n, d, seed=seed)
        S = synth.dirichlet_clusters(m, d, seed=seed, stream=1)
    else:
        d = 512
        R = synth.block_sparse_rows(n, seed=seed)
        S = synth.block_sparse_rows(m, seed=seed, stream=1)
    if self_join:
        S = R
    return rng, R, S, self_join, d


@pytest.mark.parametrize("prec", PRECS)
def test_random_indexed_joins(orc, prec):
    built = pruned = 0
    for seed in range(12):
        rng, R, S, self_join, d = draw_clustered(seed)
        n, m = len(R), len(S)
        pi, pj = synth.sample_pairs(n, m, 4000, self_join, seed=seed)
        d2 = orc.pair_d2(R, S, pi, pj)
        eps = float(np.sqrt(synth.order_statistic(d2, float(rng.choice([0.0005, 0.002, 0.01])))))
        pivots = int(rng.choice([0, 4, 16, 64]))
        ref = orc.eps_join(R, None if self_join else S, eps)
        got, info = ops.join_eps_indexed(dev(R), None if self_join else dev(S), eps, prec, pivots=pivots)
        assert_eps_equal(got, ref, d, "seed %d n %d m %d d %d self %s pivots %d eps %.9g/%s" % (
            seed, n, m, d, self_join, pivots, eps, prec))
        built += info.pivots > 0
        pruned += (info.tiles_computed < info.tiles_total or
                   info.ksteps_computed < info.tiles_computed * info.ksteps_per_tile)
    # the sweep exercises the index's pruning, not only the plain fallback
    assert built >= 6 and pruned >= 3, (built, pruned)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_random_filtered_joins(orc, prec):
    for seed in range(12):
        rng, R, S, self_join, d = draw_case(seed)
        n, m = len(R), len(S)
        if self_join and n < 2:
            continue
        nl = int(rng.integers(1, 5))
        lr = rng.integers(0, nl, size=n).astype(np.int32)
        ls = lr if self_join else rng.integers(0, nl, size=m).astype(np.int32)
        label = int(rng.integers(0, nl + 1))  # nl: a label no row has
        pi, pj = synth.sample_pairs(n, m, 4000, self_join, seed=seed)
        eps = float(np.sqrt(synth.order_statistic(orc.pair_d2(R, S, pi, pj), 0.02)))
        rr = np.nonzero(lr == label)[0]
        ss = rr if self_join else np.nonzero(ls == label)[0]
        if len(rr) and len(ss):
            ref = orc.eps_join(np.ascontiguousarray(R[rr]), None if self_join else np.ascontiguousarray(S[ss]), eps)
            ref = {"i": rr[ref["i"]], "j": ss[ref["j"]], "dist": ref["dist"], "count": ref["count"]}
        else:
            e = np.zeros(0, np.int64)
            ref = {"i": e, "j": e, "dist": np.zeros(0, np.float32), "count": 0}
        for plan in ("filter_first", "match_first"):
            got = ops.join_eps_filtered(dev(R), None if self_join else dev(S), eps, dev(lr),
                                        None if self_join else dev(ls), label, plan, prec)
            assert_eps_equal(got, ref, d, "seed %d n %d m %d d %d self %s label %d/%s/%s" % (
                seed, n, m, d, self_join, label, plan, prec))
