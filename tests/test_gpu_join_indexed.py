"""GPU parity of the index-pruned eps-join against the float64 oracle: the
same pairs, in the same order, as the plain join, while tiles that cannot
hold a result pair are skipped."""
import numpy as np
import pytest
import torch

from gpu_util import assert_eps_equal, dev, host
from paper_1812_07607_amd import ops, synth

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "bf16", "fp16", "fp8"]


def eps_quantile(orc, R, S, pairs, q):
    d2 = orc.pair_d2(R, S, pairs[0], pairs[1])
    return float(np.sqrt(synth.order_statistic(d2, q)))


@pytest.mark.parametrize("prec", PRECS)
def test_histogram_self_join_indexed(orc, prec):
    """8,000 palette-patch histograms (16 base colours): the 0.01% and 1%
    quantile self-joins; most tiles pair different colours and are pruned."""
    cfg = synth.config2(0.08)
    H = orc.hist_rgb8(cfg["patches"], 8)
    for q in (cfg["q"], 0.01):
        eps = eps_quantile(orc, H, H, cfg["pairs"], q)
        ref = orc.eps_join(H, None, eps)
        got, info = ops.join_eps_indexed(dev(H), None, eps, prec)
        assert_eps_equal(got, ref, 512, "indexed histograms q=%g/%s" % (q, prec))
        assert info.pivots > 0 and info.tiles_total == 32 * 33 // 2
        if q == cfg["q"]:
            assert info.tiles_computed < info.tiles_total // 2, info


@pytest.mark.parametrize("prec", PRECS)
def test_mixture_join_indexed(orc, prec):
    """R 3,000 x S 5,000 rows of a tight 12-centre mixture, d = 64: eps at
    several quantiles, from below the nearest pair to above the largest
    cluster diameter (every tile survives)."""
    R = synth.gaussian_mixture_unit(3000, 64, 12, sigma=0.02, seed=61)
    S = synth.gaussian_mixture_unit(5000, 64, 12, sigma=0.02, seed=61, stream=1)
    S[4321] = R[17]  # a duplicate
    pairs = synth.sample_pairs(3000, 5000, 20000, False, seed=62)
    for q in (0.0, 0.0005, 0.02, 0.2, 1.0):
        eps = eps_quantile(orc, R, S, pairs, q) if q > 0 else 0.0
        ref = orc.eps_join(R, S, eps)
        got, info = ops.join_eps_indexed(dev(R), dev(S), eps, prec)
        assert_eps_equal(got, ref, 64, "indexed mixture q=%g/%s" % (q, prec))
        assert info.tiles_computed <= info.tiles_total == 12 * 20


@pytest.mark.parametrize("prec", PRECS)
def test_block_sparse_rows_skip_ksteps(orc, prec):
    """Rows nonzero in one of 8 blocks of 64 coordinates, 10% of them faint
    (length 0.05): K-steps that are zero in every row of a tile are skipped
    and the pairs are still the oracle's.  eps = 0.12 holds every faint
    pair, whatever their blocks (products all zero); eps = 1.5 holds every
    pair of rows of different blocks (d^2 = 2 from the norms alone), so
    every tile survives, the full grid runs with the masks, and tiles of two
    different blocks run a single all-zero step."""
    R = synth.block_sparse_rows(1200, seed=71)
    S = synth.block_sparse_rows(1100, seed=71, stream=1)
    pairs = synth.sample_pairs(1200, 1100, 20000, False, seed=72)
    for eps in (0.12, eps_quantile(orc, R, S, pairs, 0.01), 1.5):
        ref = orc.eps_join(R, S, eps)
        got, info = ops.join_eps_indexed(dev(R), dev(S), eps, prec, pivots=16)
        assert_eps_equal(got, ref, 512, "block-sparse eps=%g/%s" % (eps, prec))
        assert info.ksteps_per_tile == {"fp32": 16, "bf16": 8, "fp16": 8, "fp8": 4}[prec]
        assert info.ksteps_computed < info.tiles_computed * info.ksteps_per_tile, info
    X = synth.block_sparse_rows(1500, seed=73)
    for eps in (0.12, 1.5):
        ref = orc.eps_join(X, None, eps)
        got, info = ops.join_eps_indexed(dev(X), None, eps, prec, pivots=16)
        assert_eps_equal(got, ref, 512, "block-sparse self eps=%g/%s" % (eps, prec))
        assert info.ksteps_computed < info.tiles_computed * info.ksteps_per_tile, info


def test_histogram_ksteps_skipped(orc):
    """On palette histograms ordered by pivot, a tile's rows mostly share a
    colour, and some of the 8 K-steps (64 bins, one red level, each in fp16)
    of a computed tile are zero on one side (noise spreads a patch over
    several red levels, so most steps stay)."""
    cfg = synth.config2(0.08)
    H = orc.hist_rgb8(cfg["patches"], 8)
    eps = eps_quantile(orc, H, H, cfg["pairs"], cfg["q"])
    got, info = ops.join_eps_indexed(dev(H), None, eps, "fp16")
    assert_eps_equal(got, orc.eps_join(H, None, eps), 512, "histogram ksteps")
    assert info.ksteps_per_tile == 8
    assert info.ksteps_computed < info.tiles_computed * 8, info


@pytest.mark.parametrize("shape", [(513, 1000, 1), (700, 2049, 129), (1500, 600, 300)])
def test_ragged_shapes_indexed(orc, shape):
    nR, nS, d = shape
    R = synth.gaussian_mixture_unit(nR, d, 9, seed=nR + d) if d > 1 else synth.uniform_rows(nR, 1, seed=3)
    S = synth.gaussian_mixture_unit(nS, d, 9, seed=nR + d, stream=1) if d > 1 else synth.uniform_rows(nS, 1, seed=4)
    pairs = synth.sample_pairs(nR, nS, 4000, False, seed=5)
    eps = eps_quantile(orc, R, S, pairs, 0.01)
    ref = orc.eps_join(R, S, eps)
    got, info = ops.join_eps_indexed(dev(R), dev(S), eps, "bf16", pivots=20)
    assert_eps_equal(got, ref, d, "indexed %s" % (shape,))
    assert info.pivots == 20


def test_self_join_with_duplicates_indexed(orc):
    X = synth.gaussian_mixture_unit(2600, 48, 7, sigma=0.03, seed=9)
    X[100] = X[50]
    X[2500] = X[50]
    X[1200:1210] = X[3]
    pairs = synth.sample_pairs(2600, 2600, 20000, True, seed=2)
    for eps in (0.0, eps_quantile(orc, X, X, pairs, 0.005)):
        ref = orc.eps_join(X, None, eps)
        got, info = ops.join_eps_indexed(dev(X), None, eps, "fp16")
        assert_eps_equal(got, ref, 48, "indexed self eps=%g" % eps)


def test_fallbacks_run_the_plain_join(orc):
    # infinite eps, and a relation within one 256-row tile: no index, same result
    X = synth.gaussian_mixture_unit(700, 16, 4, seed=10)
    Y = synth.gaussian_mixture_unit(200, 16, 4, seed=10, stream=1)
    ref = orc.eps_join(X, Y, float("inf"))
    got, info = ops.join_eps_indexed(dev(X), dev(Y), float("inf"), "bf16")
    assert info.pivots == 0 and got.count == 700 * 200
    assert_eps_equal(got, ref, 16, "eps = inf")
    eps = 0.3
    ref = orc.eps_join(X, Y, eps)
    got, info = ops.join_eps_indexed(dev(X), dev(Y), eps, "bf16")
    assert info.pivots == 0
    assert_eps_equal(got, ref, 16, "200-row S")


def test_full_histogram_workload_equals_plain_join():
    """100,000 patches at the 0.01% quantile: the indexed join's arrays equal
    the plain join's (which the oracle tests pin) and most tiles are pruned."""
    cfg = synth.config2(1.0)
    H = ops.featurize_rgb8(dev(cfg["patches"]), 8)
    pi, pj = cfg["pairs"]
    d2 = host(ops.pair_d2(H, H, torch.from_numpy(pi), torch.from_numpy(pj)))
    eps = float(np.sqrt(synth.order_statistic(d2, cfg["q"])))
    plain = ops.join_eps(H, None, eps, "fp16")
    got, info = ops.join_eps_indexed(H, None, eps, "fp16")
    assert got.count == plain.count > 0
    assert torch.equal(got.i, plain.i) and torch.equal(got.j, plain.j) and torch.equal(got.dist, plain.dist)
    assert info.tiles_computed < info.tiles_total // 4, info


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_index_degenerate_inputs(orc, prec):
    """All rows identical (every ball has radius 0, every tile survives, every
    pair is at distance 0), exactly two tiles per relation, and more pivots
    asked for than S has rows."""
    X = np.tile(synth.gaussian_mixture_unit(1, 40, 1, seed=91), (700, 1))
    got, info = ops.join_eps_indexed(dev(X), None, 0.0, prec)
    assert_eps_equal(got, orc.eps_join(X, None, 0.0), 40, "identical rows/%s" % prec)
    assert got.count == 700 * 699 // 2 and info.tiles_computed == info.tiles_total
    R = synth.gaussian_mixture_unit(512, 24, 5, sigma=0.02, seed=92)
    S = synth.gaussian_mixture_unit(512, 24, 5, sigma=0.02, seed=92, stream=1)
    pairs = synth.sample_pairs(512, 512, 10000, False, seed=93)
    eps = eps_quantile(orc, R, S, pairs, 0.01)
    for piv in (0, 5000):
        got, info = ops.join_eps_indexed(dev(R), dev(S), eps, prec, pivots=piv)
        assert_eps_equal(got, orc.eps_join(R, S, eps), 24, "two tiles pivots=%d/%s" % (piv, prec))
        assert info.tiles_total == 4 and 0 < info.pivots <= 512


def _two_support_clusters(seed, stream, shuffle):
    """16,384 rows of d = 256 histogram-like vectors in 8 clusters of 2,048
    rows, cluster-major unless shuffled: clusters 0-3 nonzero only in bins
    64c .. 64c + 63 (one fp16 K-step), clusters 4-7 in all 256 bins (four
    K-steps).  Each row is its cluster's centre (drawn from seed, the same
    for every stream) plus small noise (drawn from seed and stream).  With
    16 pivots at a stride of 1,024 rows of the cluster-major relation, each
    cluster holds two pivots and every tile of the pivot order one cluster."""
    c = np.random.default_rng(seed)
    cent = [c.dirichlet(np.ones(64)) for _ in range(4)] + [c.dirichlet(np.ones(256)) for _ in range(4)]
    rng = np.random.default_rng([seed, stream])
    out = np.zeros((8 * 2048, 256), np.float32)
    for k in range(8):
        rows = slice(2048 * k, 2048 * (k + 1))
        if k < 4:
            out[rows, 64 * k:64 * k + 64] = np.clip(cent[k] + rng.normal(0, 0.002, (2048, 64)), 0, None)
        else:
            out[rows] = np.clip(cent[k] + rng.normal(0, 0.001, (2048, 256)), 0, None)
    return out[rng.permutation(len(out))] if shuffle else out


_TWO_SUPPORT = {}


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_single_kstep_tiles_beside_wider_ones(orc, prec):
    """16,384 x 16,384 rows in 8 clusters whose tiles run one or four
    K-steps (2-byte formats): with 512 surviving tiles over the persistent
    workgroups,
    a workgroup's first tile often has a single K-step and its next tile
    more (the masked pass takes each tile's step count from the step it
    issued).  Equal to the oracle; the cross-cluster tiles are pruned."""
    if not _TWO_SUPPORT:
        R = _two_support_clusters(211, 0, True)
        S = _two_support_clusters(211, 1, False)
        rng = np.random.default_rng(213)
        pi, pj = rng.integers(0, len(R), 20000), rng.integers(0, len(S), 20000)
        eps = eps_quantile(orc, R, S, (pi, pj), 0.002)
        _TWO_SUPPORT.update(R=R, S=S, eps=eps, ref=orc.eps_join(R, S, eps))
    R, S, eps, ref = (_TWO_SUPPORT[k] for k in ("R", "S", "eps", "ref"))
    got, info = ops.join_eps_indexed(dev(R), dev(S), eps, prec)
    assert_eps_equal(got, ref, 256, "two-support clusters/" + prec)
    assert info.tiles_computed <= info.tiles_total // 4, info
    assert info.ksteps_computed < info.tiles_computed * info.ksteps_per_tile, info
