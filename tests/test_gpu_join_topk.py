"""GPU parity of the top-k join against the float64 oracle: every row's k
indices equal the oracle's, in order (ties to the smaller index)."""
import numpy as np
import pytest

from gpu_util import assert_topk_equal, dev, host
from paper_1812_07607_amd import ops, synth

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "bf16", "fp16", "fp8"]


@pytest.mark.parametrize("prec", PRECS)
def test_mixture_top10(orc, prec):
    """Unit-norm 1,000-centre mixture rows (sigma 0.05), d = 128, top-10."""
    R = synth.gaussian_mixture_unit(1500, 128, 50, seed=303)
    S = synth.gaussian_mixture_unit(6000, 128, 50, seed=303, stream=1)
    ref_j, _, ref_dist = orc.topk(R, S, 10)
    got = ops.join_topk(dev(R), dev(S), 10, prec=prec)
    assert_topk_equal(got, ref_j, ref_dist, 128, "mixture/" + prec)
    assert got.band_entries >= 1500 * 10


@pytest.mark.parametrize("prec", PRECS)
def test_fp8_store_shape_top32(orc, prec):
    """d = 256 queries against a store, top-32 (the FP8 workload's shape)."""
    Q = synth.gaussian_mixture_unit(300, 256, 64, seed=404, stream=1)
    S = synth.gaussian_mixture_unit(20000, 256, 64, seed=404)
    ref_j, _, ref_dist = orc.topk(Q, S, 32)
    got = ops.join_topk(dev(Q), dev(S), 32, prec=prec)
    assert_topk_equal(got, ref_j, ref_dist, 256, "store/" + prec)


@pytest.mark.parametrize("prec", PRECS)
def test_self_exclude(orc, prec):
    X = synth.gaussian_mixture_unit(900, 40, 9, seed=5)
    X[10] = X[20]
    ref_j, _, ref_dist = orc.topk(X, None, 7, exclude_self=True)
    got = ops.join_topk(dev(X), None, 7, exclude_self=True, prec=prec)
    assert_topk_equal(got, ref_j, ref_dist, 40, "self/" + prec)
    ref_j, _, ref_dist = orc.topk(X, None, 7)
    got = ops.join_topk(dev(X), None, 7, prec=prec)
    assert_topk_equal(got, ref_j, ref_dist, 40, "self-incl/" + prec)


@pytest.mark.parametrize("prec", PRECS)
def test_ties_at_kth(orc, prec):
    """Integer-grid rows: many equal distances at and inside the k-th."""
    R = synth.integer_grid_rows(200, 6, levels=3, seed=6)
    S = synth.integer_grid_rows(700, 6, levels=3, seed=6, stream=1)
    for k in (1, 5, 16):
        ref_j, _, ref_dist = orc.topk(R, S, k)
        got = ops.join_topk(dev(R), dev(S), k, prec=prec)
        assert_topk_equal(got, ref_j, ref_dist, 6, "grid k=%d/%s" % (k, prec))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(1, 1, 1, 1), (5, 3, 7, 10), (300, 40, 33, 64), (257, 513, 130, 3)])
def test_ragged_and_padding(orc, prec, shape):
    nR, nS, d, k = shape
    R = synth.uniform_rows(nR, d, seed=nR)
    S = synth.uniform_rows(nS, d, seed=nR, stream=1)
    ref_j, _, ref_dist = orc.topk(R, S, k)
    got = ops.join_topk(dev(R), dev(S), k, prec=prec)
    assert_topk_equal(got, ref_j, ref_dist, d, "%s/%s" % (shape, prec))


def test_small_band_capacity_retry(orc):
    R = synth.gaussian_mixture_unit(100, 16, 2, seed=8)
    S = synth.gaussian_mixture_unit(5000, 16, 2, seed=8, stream=1)
    ref_j, _, ref_dist = orc.topk(R, S, 200)
    got = ops.join_topk(dev(R), dev(S), 200, prec="fp8", band_cap=512)
    assert_topk_equal(got, ref_j, ref_dist, 16, "k=200 fp8")


def test_histogram_topk(orc):
    cfg = synth.config2(0.03)
    H = orc.hist_rgb8(cfg["patches"], 8)
    ref_j, _, ref_dist = orc.topk(H, None, 5, exclude_self=True)
    got = ops.join_topk(dev(H), None, 5, exclude_self=True, prec="fp16")
    assert_topk_equal(got, ref_j, ref_dist, 512, "histograms")
    assert got.ties == 0  # exact on the 2^-10 grid: no float64 needed


@pytest.mark.parametrize("k", [10, 64])
def test_many_splits_large_union(orc, k):
    """Few query rows against a long S: the work is split over hundreds of S
    ranges, so a row's union of band buffers holds thousands of entries (k =
    10: it is filtered down to registers; k = 64: it stays in memory)."""
    R = synth.gaussian_mixture_unit(50, 32, 40, seed=31)
    S = synth.gaussian_mixture_unit(60000, 32, 40, seed=31, stream=1)
    ref_j, _, ref_dist = orc.topk(R, S, k)
    got = ops.join_topk(dev(R), dev(S), k, prec="bf16")
    assert_topk_equal(got, ref_j, ref_dist, 32, "splits k=%d" % k)


def test_fp8_top32_seeded_by_bf16_pilot(orc):
    """The E4M3 top-32 on a 4,096-centre d = 256 store (the FP8 workload at
    a tenth of its size: 400,000 store rows, 5,000 queries).  Unseeded, the
    E4M3 band keeps most unrelated rows until a row has met 32 neighbours
    and overflows any buffer; the bf16 pilot over every 16th store row seeds
    it.  The oracle checks 64 sampled query rows (rows of a top-k join are
    independent)."""
    cfg = synth.config4(0.1)
    S, Q = cfg["S"], cfg["Q"]
    got = ops.join_topk(dev(Q), dev(S), 32, prec="fp8")
    rows = synth.sample_rows(Q.shape[0], 64, seed=12)
    ref_j, _, ref_dist = orc.topk(np.ascontiguousarray(Q[rows]), S, 32)
    sub = ops.TopkResult(got.j[dev(rows).long()], got.dist[dev(rows).long()], 0, 0)
    assert_topk_equal(sub, ref_j, ref_dist, 256, "fp8 store top-32, sampled rows")
    # the band stays near the 32 nearest (plus the E4M3 margin's contenders)
    assert got.band_entries < Q.shape[0] * 2000


def test_many_exact_ties_use_the_large_selection(orc):
    """300 copies of one row in S, all at the same distance from every query
    row: more near-tie contenders than the small selection holds (256), so
    the library selects again with the large one (512); ties go to the
    smaller index."""
    rng = np.random.default_rng(77)
    S = rng.standard_normal((3000, 48)).astype(np.float32)
    S[1000:1300] = S[5]
    R = (S[5] + 0.01 * rng.standard_normal((40, 48))).astype(np.float32)
    ref_j, _, ref_dist = orc.topk(R, S, 10)
    got = ops.join_topk(dev(R), dev(S), 10, prec="bf16")
    assert_topk_equal(got, ref_j, ref_dist, 48, "300 exact ties")


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_more_exact_ties_than_the_selection_holds(orc, prec):
    """1,000 copies of one row in S: every query row has 1,000 contenders at
    its k-th distance, more than the selection holds in LDS (512), so those
    rows are selected over their band buffers in memory; ties go to the
    smaller index.  A second query set keeps only some rows on the ties."""
    rng = np.random.default_rng(78)
    S = rng.standard_normal((6000, 40)).astype(np.float32)
    S[2000:3000] = S[7]
    R = (S[7] + 0.01 * rng.standard_normal((24, 40))).astype(np.float32)
    R[10:] = rng.standard_normal((14, 40)).astype(np.float32)  # rows far from the copies
    for k in (10, 200):
        ref_j, _, ref_dist = orc.topk(R, S, k)
        got = ops.join_topk(dev(R), dev(S), k, prec=prec)
        assert_topk_equal(got, ref_j, ref_dist, 40, "1,000 exact ties k=%d/%s" % (k, prec))
