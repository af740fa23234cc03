"""The label filter before or after the match (the plan-order experiment):
both plans give the pairs of the oracle's join restricted to rows with the
label, in (i, j) order."""
import numpy as np
import pytest
import torch

from gpu_util import assert_eps_equal, dev
from paper_1812_07607_amd import ops, synth

pytestmark = pytest.mark.gpu


def restricted_oracle(orc, R, S, lab_r, lab_s, label, eps, self_join):
    """Oracle join of the rows with the label; indices of the full relations."""
    rr = np.nonzero(lab_r == label)[0]
    ss = rr if self_join else np.nonzero(lab_s == label)[0]
    if len(rr) == 0 or len(ss) == 0:
        e = np.zeros(0, np.int64)
        return {"i": e, "j": e, "dist": np.zeros(0, np.float32), "count": 0}
    if self_join:
        ref = orc.eps_join(np.ascontiguousarray(R[rr]), None, eps)
        return {"i": rr[ref["i"]], "j": rr[ref["j"]], "dist": ref["dist"], "count": ref["count"]}
    ref = orc.eps_join(np.ascontiguousarray(R[rr]), np.ascontiguousarray(S[ss]), eps)
    return {"i": rr[ref["i"]], "j": ss[ref["j"]], "dist": ref["dist"], "count": ref["count"]}


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_histogram_self_join_both_plans(orc, prec):
    cfg = synth.config2(0.05)
    H = orc.hist_rgb8(cfg["patches"], 8)
    labels = cfg["colour"].astype(np.int32)  # the palette colour stands in for a detector's label
    pairs = cfg["pairs"]
    eps = float(np.sqrt(synth.order_statistic(orc.pair_d2(H, H, *pairs), 0.001)))
    for label in (3, 11):
        ref = restricted_oracle(orc, H, None, labels, None, label, eps, True)
        for plan in ("filter_first", "match_first"):
            got = ops.join_eps_filtered(dev(H), None, eps, dev(labels), None, label, plan, prec)
            assert_eps_equal(got, ref, 512, "%s label %d/%s" % (plan, label, prec))


def test_two_relations_both_plans(orc):
    R = synth.gaussian_mixture_unit(2500, 64, 10, seed=71)
    S = synth.gaussian_mixture_unit(3100, 64, 10, seed=71, stream=1)
    rng = np.random.default_rng(72)
    lr = rng.integers(0, 4, size=2500).astype(np.int32)
    ls = rng.integers(0, 4, size=3100).astype(np.int32)
    pairs = synth.sample_pairs(2500, 3100, 20000, False, seed=73)
    eps = float(np.sqrt(synth.order_statistic(orc.pair_d2(R, S, *pairs), 0.01)))
    for label in (0, 2, 9):  # 9: no row has it
        ref = restricted_oracle(orc, R, S, lr, ls, label, eps, False)
        res = [ops.join_eps_filtered(dev(R), dev(S), eps, dev(lr), dev(ls), label, plan, "bf16")
               for plan in ("filter_first", "match_first")]
        for got, plan in zip(res, ("filter_first", "match_first")):
            assert_eps_equal(got, ref, 64, "%s label %d" % (plan, label))
        assert torch.equal(res[0].i, res[1].i) and torch.equal(res[0].j, res[1].j)


def test_plans_degenerate_labels(orc):
    """Every row labelled (both plans are the plain join), one labelled row
    (a self-join has no pair; a two-relation join one row against the
    labelled S rows), and a self-join whose labelled rows are all identical."""
    X = synth.gaussian_mixture_unit(1800, 32, 6, sigma=0.03, seed=81)
    pairs = synth.sample_pairs(1800, 1800, 20000, True, seed=82)
    eps = float(np.sqrt(synth.order_statistic(orc.pair_d2(X, X, *pairs), 0.01)))
    every = np.full(1800, 5, np.int32)
    plain = ops.join_eps(dev(X), None, eps, "bf16")
    for plan in ("filter_first", "match_first"):
        got = ops.join_eps_filtered(dev(X), None, eps, dev(every), None, 5, plan, "bf16")
        assert got.count == plain.count and torch.equal(got.i, plain.i) and torch.equal(got.j, plain.j), plan
    one = np.zeros(1800, np.int32)
    one[977] = 1
    for plan in ("filter_first", "match_first"):
        got = ops.join_eps_filtered(dev(X), None, eps, dev(one), None, 1, plan, "fp16")
        assert got.count == 0, plan
        got = ops.join_eps_filtered(dev(X), dev(X), eps, dev(one), dev(every - 4), 1, plan, "fp16")
        ref = restricted_oracle(orc, X, X, one, every - 4, 1, eps, False)
        assert_eps_equal(got, ref, 32, "one row/%s" % plan)
    Y = X.copy()
    lab = (np.arange(1800) % 3 == 0).astype(np.int32)
    Y[lab == 1] = Y[0]
    for plan in ("filter_first", "match_first"):
        got = ops.join_eps_filtered(dev(Y), None, 0.0, dev(lab), None, 1, plan, "bf16")
        ref = restricted_oracle(orc, Y, None, lab, None, 1, 0.0, True)
        assert_eps_equal(got, ref, 32, "identical rows/%s" % plan)
        assert got.count == 600 * 599 // 2
