"""Adversarial inputs for the margin-widened candidate filter.

Every input value sits just below half a unit in the last place of the
candidate format above a representable value, with the same sign
everywhere, so every rounding residual of the operand copy has the same
sign and the error of the low-precision dot product is as large as its
Cauchy-Schwarz bound allows.  eps is then set exactly at a pair's canonical
distance (the pair is in) and one double below it (the pair is out).  A pair
missing from the candidates would be missing from the output, so equality
with the float64 oracle means no misses."""
import numpy as np
import pytest

from gpu_util import assert_eps_equal, assert_topk_equal, dev
from paper_1812_07607_amd import ops

pytestmark = pytest.mark.gpu


def _exp2(x):
    return np.floor(np.log2(np.abs(x))).astype(np.int64)


def aligned_rows(fmt, n, d, seed):
    """n x d float32 rows whose residuals against the `fmt` operand copy all
    have the same sign (+0.49 of the format's unit in the last place)."""
    rng = np.random.default_rng(seed)
    if fmt == "bf16":
        v = (0.25 + rng.random((n, d))).astype(np.float32)
        b = v.view(np.uint32)
        g = (((b + np.uint32(0x7FFF) + ((b >> 16) & 1)) >> 16) << 16).view(np.float32)
        ulp = np.exp2(_exp2(g) - 7)
    elif fmt == "fp16":
        v = 0.25 + rng.random((n, d))
        g = v.astype(np.float16).astype(np.float32)
        ulp = np.exp2(_exp2(g) - 10)
    elif fmt == "fp8":
        # E4M3 values (1 + m/8) 2^e with e in [-3, 7], times a row scale 2^-8;
        # element 0 is 288 * 2^-8 so the row's scale is exactly 2^-8
        e = rng.integers(-3, 8, size=(n, d))
        m = rng.integers(0, 8, size=(n, d))
        y = (1.0 + m / 8.0) * np.exp2(e)
        y[:, 0] = 288.0
        g = (y * 2.0 ** -8).astype(np.float32)
        ulp = np.exp2(_exp2(y) - 3) * 2.0 ** -8
    else:  # fp32: no operand rounding; a wide range of magnitudes stresses the accumulation
        v = np.exp2(rng.uniform(-6, 4, size=(n, d))) * (1 + rng.random((n, d)))
        return v.astype(np.float32)
    x = (g.astype(np.float64) + 0.49 * ulp).astype(np.float32)
    return x


def boundary_eps(orc, R, S, qs):
    """eps values exactly at the canonical distance of pairs at the given
    quantiles of all pair distances, and the double just below each."""
    pi, pj = np.meshgrid(np.arange(R.shape[0]), np.arange(S.shape[0]), indexing="ij")
    d2 = orc.pair_d2(R, S, pi.ravel(), pj.ravel())
    srt = np.sort(d2)
    out = []
    for q in qs:
        e = float(np.sqrt(srt[max(0, int(q * len(srt)) - 1)]))
        out += [e, float(np.nextafter(e, 0.0))]
    return out


FORMATS = ["bf16", "fp16", "fp8", "fp32"]


@pytest.mark.parametrize("fmt", FORMATS)
def test_aligned_residuals_eps_at_pair_distances(orc, fmt):
    d = 96
    R = aligned_rows(fmt, 300, d, seed=11)
    S = aligned_rows(fmt, 420, d, seed=12)
    S[7] = R[3]  # a duplicate: distance 0 stays in at every eps
    for eps in boundary_eps(orc, R, S, [0.0005, 0.005, 0.05]):
        ref = orc.eps_join(R, S, eps)
        got = ops.join_eps(dev(R), dev(S), eps, fmt)
        assert_eps_equal(got, ref, d, "aligned %s eps=%r" % (fmt, eps))
        assert got.candidates >= got.count


@pytest.mark.parametrize("fmt", FORMATS)
def test_aligned_residuals_self_join(orc, fmt):
    d = 64
    X = aligned_rows(fmt, 520, d, seed=13)
    X[300] = X[17]
    for eps in boundary_eps(orc, X[:200], X, [0.001, 0.02]):
        ref = orc.eps_join(X, None, eps)
        got = ops.join_eps(dev(X), None, eps, fmt)
        assert_eps_equal(got, ref, d, "aligned self %s eps=%r" % (fmt, eps))


@pytest.mark.parametrize("fmt", FORMATS)
def test_aligned_residuals_topk(orc, fmt):
    d = 80
    R = aligned_rows(fmt, 260, d, seed=14)
    S = aligned_rows(fmt, 3000, d, seed=15)
    S[100:110] = S[5]  # ten exact ties
    for k in (1, 10, 33):
        ref_j, _, ref_dist = orc.topk(R, S, k)
        got = ops.join_topk(dev(R), dev(S), k, prec=fmt)
        assert_topk_equal(got, ref_j, ref_dist, d, "aligned top-%d %s" % (k, fmt))
