"""GPU parity of the index-pruned top-k join: every row's k indices equal
the oracle's, in order (ties to the smaller index), and equal the plain
top-k join's, while tiles that cannot hold a row's k nearest are skipped."""
import numpy as np
import pytest
import torch

from gpu_util import assert_topk_equal, dev
from paper_1812_07607_amd import ops, synth

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "bf16", "fp16", "fp8"]


@pytest.mark.parametrize("prec", PRECS)
def test_mixture_topk_indexed(orc, prec):
    """R 4,096 x S 6,144 rows of a tight 4-centre mixture, d = 64: k = 1,
    10 and 32; tiles that pair different clusters are skipped."""
    R = synth.gaussian_mixture_unit(4096, 64, 4, sigma=0.02, seed=161)
    S = synth.gaussian_mixture_unit(6144, 64, 4, sigma=0.02, seed=161, stream=1)
    S[4321] = R[17]  # a duplicate
    for k in (1, 10, 32):
        ref_j, _, ref_dist = orc.topk(R, S, k)
        got, info = ops.join_topk_indexed(dev(R), dev(S), k, prec=prec)
        assert_topk_equal(got, ref_j, ref_dist, 64, "mixture k=%d/%s" % (k, prec))
        assert info.pivots > 0 and info.tiles_total == 16 * 24
        assert info.tiles_computed < info.tiles_total, info


@pytest.mark.parametrize("prec", PRECS)
def test_self_join_topk_indexed(orc, prec):
    """A self-join with and without the row itself, duplicates planted (exact
    ties at distance 0 and at the k-th), 6,000 rows of a 3-centre mixture."""
    X = synth.gaussian_mixture_unit(6000, 32, 3, sigma=0.02, seed=171)
    X[100:110] = X[5]
    for excl in (True, False):
        ref_j, _, ref_dist = orc.topk(X, None, 10, exclude_self=excl)
        got, info = ops.join_topk_indexed(dev(X), None, 10, exclude_self=excl, prec=prec)
        assert_topk_equal(got, ref_j, ref_dist, 32, "self excl=%s/%s" % (excl, prec))
        assert info.tiles_computed < info.tiles_total, info


def test_histogram_topk_indexed_equals_plain(orc):
    """8,000 palette-patch histograms (fp16 candidates, the exact format on
    them): the pruned and the plain top-5 self-joins are identical and equal
    to the oracle's; tiles and K-steps are skipped."""
    cfg = synth.config2(0.08)
    H = orc.hist_rgb8(cfg["patches"], 8)
    ref_j, _, ref_dist = orc.topk(H, None, 5, exclude_self=True)
    got, info = ops.join_topk_indexed(dev(H), None, 5, exclude_self=True, prec="fp16")
    plain = ops.join_topk(dev(H), None, 5, exclude_self=True, prec="fp16")
    assert_topk_equal(got, ref_j, ref_dist, 512, "histograms")
    assert torch.equal(got.j, plain.j) and torch.equal(got.dist, plain.dist)
    assert info.tiles_computed < 0.7 * info.tiles_total, info
    # bins empty in every row of a pivot-ordered tile drop out of its K-steps
    assert 0 < info.ksteps_computed < info.tiles_computed * info.ksteps_per_tile, info


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_ties_and_small_relations(orc, prec):
    """Integer-grid rows (many equal distances at the k-th), the pivot count
    given, and a relation of a single tile (the plain join runs)."""
    R = synth.integer_grid_rows(700, 6, levels=3, seed=181)
    S = synth.integer_grid_rows(900, 6, levels=3, seed=181, stream=1)
    for k, piv in ((5, 0), (16, 8)):
        ref_j, _, ref_dist = orc.topk(R, S, k)
        got, info = ops.join_topk_indexed(dev(R), dev(S), k, prec=prec, pivots=piv)
        assert_topk_equal(got, ref_j, ref_dist, 6, "grid k=%d/%s" % (k, prec))
    small = synth.gaussian_mixture_unit(200, 16, 4, seed=182)
    ref_j, _, ref_dist = orc.topk(small, None, 3, exclude_self=True)
    got, info = ops.join_topk_indexed(dev(small), None, 3, exclude_self=True, prec=prec)
    assert_topk_equal(got, ref_j, ref_dist, 16, "single tile/" + prec)
    assert info.pivots == 0 and info.tiles_computed == info.tiles_total


@pytest.mark.parametrize("prec", PRECS)
def test_random_topk_indexed_sweep(orc, prec):
    """Seeded clustered relations of 257..4,000 rows and 2..6 centres, random
    k, self-joins with and without the row itself: equal to the oracle; the
    index prunes in most of them."""
    pruned = 0
    for seed in range(10):
        rng = np.random.default_rng(9700 + seed)
        n = int(rng.integers(257, 4000))
        self_join = bool(rng.random() < 0.5)
        m = n if self_join else int(rng.integers(257, 4000))
        d = int(rng.choice([16, 64, 128]))
        c = int(rng.integers(2, 7))
        R = synth.gaussian_mixture_unit(n, d, c, sigma=0.02, seed=seed)
        S = R if self_join else synth.gaussian_mixture_unit(m, d, c, sigma=0.02, seed=seed, stream=1)
        k = int(rng.integers(1, 41))
        excl = self_join and bool(rng.random() < 0.5)
        ref_j, _, ref_dist = orc.topk(R, None if self_join else S, k, exclude_self=excl)
        got, info = ops.join_topk_indexed(dev(R), None if self_join else dev(S), k, exclude_self=excl, prec=prec)
        assert_topk_equal(got, ref_j, ref_dist, d, "seed %d n %d m %d d %d k %d self %s excl %s/%s" % (
            seed, n, m, d, k, self_join, excl, prec))
        pruned += info.tiles_computed < info.tiles_total
    assert pruned >= 4, pruned


def test_histogram_100k_topk_indexed_equals_plain(orc):
    """100,000 palette-patch histograms, the top-10 self-join without the row
    itself: the pruned join (with K-step masks; among its work items some
    whose first tile has a single K-step) equals the plain join row for row,
    and 64 seeded rows equal the oracle's."""
    cfg = synth.config2(1.0)
    hist = ops.featurize_rgb8(torch.from_numpy(cfg["patches"]).cuda(), 8)
    ref = ops.join_topk(hist, None, 10, exclude_self=True, prec="fp16")
    got, info = ops.join_topk_indexed(hist, None, 10, exclude_self=True, prec="fp16")
    bad = torch.nonzero((got.j != ref.j).any(1) | (got.dist != ref.dist).any(1)).flatten()
    assert bad.numel() == 0, "%d rows differ from the plain join, first %d" % (bad.numel(), int(bad[0]))
    assert info.tiles_computed < info.tiles_total // 2, info
    assert info.ksteps_computed < info.tiles_computed * info.ksteps_per_tile, info
    H = hist.cpu().numpy()
    rows = synth.sample_rows(H.shape[0], 64, seed=191)
    oj, _, od = orc.topk(H[rows], H, 11)
    keep = oj != np.asarray(rows)[:, None]  # the row itself, wherever it falls
    ref_j = np.stack([oj[r][keep[r]][:10] for r in range(len(rows))])
    ref_d = np.stack([od[r][keep[r]][:10] for r in range(len(rows))])
    sub = type(got)(got.j[torch.from_numpy(np.asarray(rows)).cuda()], got.dist[torch.from_numpy(np.asarray(rows)).cuda()],
                    0, 0)
    assert_topk_equal(sub, ref_j, ref_d, 512, "100k histograms, seeded rows")
