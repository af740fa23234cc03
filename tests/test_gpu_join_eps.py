"""GPU parity of the eps-join against the float64 oracle.

The emitted (i, j) pairs must equal the oracle's in content and order for
every operand format; distances within the float32 bound (gpu_util)."""
import math

import numpy as np
import pytest
import torch

from gpu_util import assert_eps_equal, dev, host
from paper_1812_07607_amd import ops, synth
from paper_1812_07607_amd._lib import DL_ERR_INVALID, DLError

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "bf16", "fp16", "fp8"]


def eps_quantile(orc, R, S, pairs, q):
    d2 = orc.pair_d2(R, S, pairs[0], pairs[1])
    return float(np.sqrt(synth.order_statistic(d2, q)))


@pytest.mark.parametrize("prec", PRECS)
def test_plain_eps_join_2000(orc, prec):
    """R, S: 2,000 x 64 L1-normalised Dirichlet-cluster vectors; eps = 0.1%
    order statistic of 10,000 sampled pair distances."""
    cfg = synth.config1(1.0)
    R, S = cfg["R"], cfg["S"]
    eps = eps_quantile(orc, R, S, cfg["pairs"], cfg["q"])
    ref = orc.eps_join(R, S, eps)
    got = ops.join_eps(dev(R), dev(S), eps, prec)
    assert_eps_equal(got, ref, 64, "config1/" + prec)
    assert got.candidates >= got.count


@pytest.mark.parametrize("prec", PRECS)
def test_histogram_self_join(orc, prec):
    """Featurise 6,000 palette patches on the GPU, then the eps self-join at
    the 0.01% order statistic, against the oracle's histograms and join."""
    cfg = synth.config2(0.06)
    H = host(ops.featurize_rgb8(dev(cfg["patches"]), 8))
    Href = orc.hist_rgb8(cfg["patches"], 8)
    assert np.array_equal(H, Href)
    eps = eps_quantile(orc, Href, Href, cfg["pairs"], cfg["q"])
    ref = orc.eps_join(Href, None, eps)
    got = ops.join_eps(dev(H), None, eps, prec)
    assert_eps_equal(got, ref, 512, "config2-small/" + prec)
    if prec == "fp16":
        # histogram entries are k/1024: the fp16 pass is exact, so the
        # candidates are exactly the result
        assert got.candidates == got.count


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 300, 3), (257, 300, 3), (300, 257, 129), (513, 700, 64),
                                   (64, 64, 256), (100, 1000, 200), (200, 333, 1024)])
def test_ragged_shapes(orc, prec, shape):
    nR, nS, d = shape
    R = synth.gaussian_mixture_unit(nR, d, 7, seed=nR + d)
    S = synth.gaussian_mixture_unit(nS, d, 7, seed=nR + d, stream=1)
    if nR > 3 and nS > 5:
        S[5] = R[3]  # a planted duplicate
    pairs = synth.sample_pairs(nR, nS, 2000, False, seed=1)
    eps = eps_quantile(orc, R, S, pairs, 0.05)
    ref = orc.eps_join(R, S, eps)
    got = ops.join_eps(dev(R), dev(S), eps, prec)
    assert_eps_equal(got, ref, d, "%s/%s" % (shape, prec))


@pytest.mark.parametrize("prec", PRECS)
def test_self_join_ragged(orc, prec):
    X = synth.gaussian_mixture_unit(777, 48, 5, seed=9)
    X[100] = X[50]
    X[700] = X[50]
    pairs = synth.sample_pairs(777, 777, 5000, True, seed=2)
    eps = eps_quantile(orc, X, X, pairs, 0.02)
    ref = orc.eps_join(X, None, eps)
    got = ops.join_eps(dev(X), None, eps, prec)
    assert_eps_equal(got, ref, 48, "self/" + prec)


@pytest.mark.parametrize("prec", PRECS)
def test_eps_zero_and_infinity(orc, prec):
    R = synth.uniform_rows(90, 20, seed=4)
    S = synth.uniform_rows(130, 20, seed=4, stream=1)
    S[[3, 77, 129]] = R[[10, 10, 89]]
    for eps in (0.0, math.inf):
        ref = orc.eps_join(R, S, eps)
        got = ops.join_eps(dev(R), dev(S), eps, prec)
        assert_eps_equal(got, ref, 20, "eps=%g/%s" % (eps, prec))
    assert ops.join_eps(dev(R), None, math.inf, prec).count == 90 * 89 // 2


@pytest.mark.parametrize("prec", PRECS)
def test_ties_on_the_boundary(orc, prec):
    """Integer-grid rows: many pairs sit exactly at eps."""
    R = synth.integer_grid_rows(400, 16, levels=3, seed=5)
    S = synth.integer_grid_rows(500, 16, levels=3, seed=5, stream=1)
    for eps in (0.5, math.sqrt(0.375), 1.0):  # d2 values on the grid are multiples of 1/16
        ref = orc.eps_join(R, S, eps)
        got = ops.join_eps(dev(R), dev(S), eps, prec)
        assert_eps_equal(got, ref, 16, "grid eps=%g/%s" % (eps, prec))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("scale", [1e-30, 1e-3, 1e3, 1e15])
def test_magnitudes(orc, prec, scale):
    R = (synth.gaussian_mixture_unit(200, 32, 4, seed=6) * np.float32(scale)).astype(np.float32)
    S = (synth.gaussian_mixture_unit(300, 32, 4, seed=6, stream=1) * np.float32(scale)).astype(np.float32)
    pairs = synth.sample_pairs(200, 300, 3000, False, seed=3)
    eps = eps_quantile(orc, R, S, pairs, 0.05)
    ref = orc.eps_join(R, S, eps)
    got = ops.join_eps(dev(R), dev(S), eps, prec)
    assert_eps_equal(got, ref, 32, "scale %g/%s" % (scale, prec))


def test_strided_rows(orc):
    big = synth.gaussian_mixture_unit(300, 80, 5, seed=7)
    R, S = big[:, :50], big[::2, 10:60]
    Rc, Sc = np.ascontiguousarray(R), np.ascontiguousarray(S)
    pairs = synth.sample_pairs(300, 150, 3000, False, seed=4)
    eps = eps_quantile(orc, Rc, Sc, pairs, 0.05)
    ref = orc.eps_join(Rc, Sc, eps)
    tb = dev(big)
    got = ops.join_eps(tb[:, :50], tb[::2, 10:60], eps, "bf16")
    assert_eps_equal(got, ref, 50, "strided")


def test_empty_relations(orc):
    R = synth.uniform_rows(10, 8, seed=1)
    E = np.zeros((0, 8), np.float32)
    assert ops.join_eps(dev(E), dev(R), 1.0).count == 0
    assert ops.join_eps(dev(R), dev(E), 1.0).count == 0
    assert ops.join_eps(dev(E), None, 1.0).count == 0


def test_out_of_float32_range_rejected():
    """Rows whose squared norms overflow float32 cannot be matched in float32."""
    R = synth.uniform_rows(10, 8, seed=1) * np.float32(1e30)
    with pytest.raises(DLError):
        ops.join_eps(dev(R), None, 1e30)


def test_non_finite_rejected():
    R = synth.uniform_rows(10, 8, seed=1)
    R[3, 2] = np.nan
    with pytest.raises(DLError):
        ops.join_eps(dev(R), None, 0.5)
    R[3, 2] = np.inf
    with pytest.raises(DLError):
        ops.join_eps(dev(R), dev(synth.uniform_rows(5, 8, seed=2)), 0.5)


def test_capacity_and_workspace_retry(orc):
    R = synth.uniform_rows(300, 6, seed=8)
    ref = orc.eps_join(R, None, 0.9)
    got = ops.join_eps(dev(R), None, 0.9, "bf16", max_candidates=16, capacity=3)
    assert_eps_equal(got, ref, 6, "retry")


def test_pair_d2_bit_exact(orc):
    R = synth.gaussian_mixture_unit(500, 100, 5, seed=1)
    S = synth.uniform_rows(400, 100, seed=1)
    pi, pj = synth.sample_pairs(500, 400, 20000, False, seed=9)
    got = host(ops.pair_d2(dev(R), dev(S), torch.from_numpy(pi), torch.from_numpy(pj)))
    assert np.array_equal(got, orc.pair_d2(R, S, pi, pj))
    with pytest.raises(DLError):
        ops.pair_d2(dev(R), dev(S), torch.tensor([0, 500]), torch.tensor([0, 0]))


def test_full_size_histogram_self_join_sampled_rows(orc):
    """100,000 patches featurised and self-joined at full size, in the
    configuration the benchmark times; the oracle checks 256 sampled rows
    (rows of an eps-join are independent, so a sampled row is an exact
    check of everything emitted for it)."""
    cfg = synth.config2(1.0)
    H = ops.featurize_rgb8(dev(cfg["patches"]), 8)
    Hn = host(H)
    eps = float(np.sqrt(synth.order_statistic(orc.pair_d2(Hn, Hn, *cfg["pairs"]), cfg["q"])))
    got = ops.join_eps(H, None, eps, "fp16")
    rows = synth.sample_rows(Hn.shape[0], 256, seed=11)
    ref = orc.eps_join(np.ascontiguousarray(Hn[rows]), Hn, eps, self_join=True, row_ids=rows)
    gi = host(got.i).astype(np.int64)
    sel = np.isin(gi, rows)
    sub = ops.EpsResult(got.i[torch.from_numpy(sel).cuda()], got.j[torch.from_numpy(sel).cuda()],
                        got.dist[torch.from_numpy(sel).cuda()], int(sel.sum()), 0, 0)
    assert_eps_equal(sub, ref, 512, "config2-full-sampled")
    # i < j everywhere and canonical order overall
    gj = host(got.j).astype(np.int64)
    assert np.all(gi < gj)
    key = gi * (1 << 20) + gj
    assert np.all(np.diff(key) > 0)


class _Misaligned(ops.Workspace):
    """A workspace whose buffer starts 16 bytes past an allocation."""

    def get(self, nbytes):
        return super().get(int(nbytes) + 256)[16:]


def test_rejects_misaligned_workspace():
    R = dev(synth.uniform_rows(300, 64, seed=11))
    with pytest.raises(DLError) as e:
        ops.join_eps(R, None, 0.5, "bf16", workspace=_Misaligned(R.device))
    assert e.value.status == DL_ERR_INVALID
    with pytest.raises(DLError) as e:
        ops.join_topk(R, R, 5, prec="bf16", workspace=_Misaligned(R.device))
    assert e.value.status == DL_ERR_INVALID


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_long_rows_keep_j_order(orc, prec):
    """Rows of 0 to ~70,000 pairs: the output ordering ranks short rows in
    registers and long ones through bitmap windows of 32,768 j values, so a
    70,000-column S with eps at the 40% order statistic spans several windows
    per row, and a far-away row yields few or no pairs."""
    R = synth.gaussian_mixture_unit(5, 8, 3, seed=41)
    S = synth.gaussian_mixture_unit(70000, 8, 3, seed=41, stream=1)
    R[4] = -R[0]  # likely far from most of S
    pairs = synth.sample_pairs(5, 70000, 4000, False, seed=3)
    eps = eps_quantile(orc, R, S, pairs, 0.4)
    ref = orc.eps_join(R, S, eps)
    got = ops.join_eps(dev(R), dev(S), eps, prec)
    assert_eps_equal(got, ref, 8, "long-rows/" + prec)


def test_rows_with_gaps_between_j_windows(orc):
    """A row of 3,000 pairs whose j values sit in two runs 190,000 apart
    (the ordering skips the empty bitmap windows between them), next to
    rows of a few hundred pairs (ranked pair against pair in LDS)."""
    R = synth.gaussian_mixture_unit(6, 8, 3, seed=43)
    S = synth.gaussian_mixture_unit(200000, 8, 3, seed=43, stream=1)
    rng = np.random.default_rng(44)
    for lo, hi, src in ((0, 1500, 0), (198500, 200000, 0), (50000, 50250, 1), (120000, 120200, 2)):
        x = R[src].astype(np.float64) + 1e-3 * rng.standard_normal((hi - lo, 8))
        S[lo:hi] = (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)
    eps = 0.01
    ref = orc.eps_join(R, S, eps)
    counts = np.bincount(ref["i"], minlength=6)
    assert counts[0] >= 3000 and 64 < counts[1] <= 256 and 64 < counts[2] <= 256
    got = ops.join_eps(dev(R), dev(S), eps, "bf16")
    assert_eps_equal(got, ref, 8, "gapped-rows")
