"""Pins for the oracle's top-k join (query q1, section "Queries": the closest
image to a query image).  Checked against a hand example, a full
lexicographic sort by numpy, and the relation to the eps-join."""
import numpy as np
import pytest

from conftest import read_golden
from paper_1812_07607_amd import synth


def full_sort_reference(orc, R, S, k, exclude_self=False):
    nR, nS = R.shape[0], S.shape[0]
    pi = np.repeat(np.arange(nR), nS)
    pj = np.tile(np.arange(nS), nR)
    d2 = orc.pair_d2(R, S, pi, pj).reshape(nR, nS)
    out_j = np.full((nR, k), -1, np.int64)
    out_d = np.full((nR, k), np.inf)
    for i in range(nR):
        js = np.arange(nS)
        dd = d2[i]
        if exclude_self:
            keep = js != i
            js, dd = js[keep], dd[keep]
        order = np.lexsort((js, dd))  # primary d2, then j
        m = min(k, len(order))
        out_j[i, :m] = js[order[:m]]
        out_d[i, :m] = dd[order[:m]]
    return out_j, out_d


def test_hand_ties(orc):
    rows = read_golden("topk_hand.txt")
    R = np.array([list(map(float, r[1:])) for r in rows if r[0] == "R"], np.float32)
    S = np.array([list(map(float, r[1:])) for r in rows if r[0] == "S"], np.float32)
    for r in rows:
        if r[0] == "k":
            k = int(r[1])
            expect = list(map(int, r[3:]))
            j, d2, dist = orc.topk(R, S, k)
            assert j[0].tolist() == expect
            assert all(np.isinf(dist[0][len([e for e in expect if e >= 0]):]))


@pytest.mark.parametrize("k", [1, 5, 10, 64])
@pytest.mark.parametrize("gen", ["mixture", "grid"])
def test_equals_first_k_of_full_sort(orc, k, gen):
    if gen == "mixture":
        R = synth.gaussian_mixture_unit(30, 12, 5, seed=1)
        S = synth.gaussian_mixture_unit(50, 12, 5, seed=1, stream=1)
    else:  # many exact ties
        R = synth.integer_grid_rows(30, 4, seed=2)
        S = synth.integer_grid_rows(50, 4, seed=2, stream=1)
    j, d2, _ = orc.topk(R, S, k)
    rj, rd = full_sort_reference(orc, R, S, k)
    assert np.array_equal(j, rj) and np.array_equal(d2, rd)


def test_top_all_is_full_sort_and_padding(orc):
    R = synth.uniform_rows(6, 3, seed=3)
    S = synth.uniform_rows(9, 3, seed=3, stream=1)
    j, d2, dist = orc.topk(R, S, 12)
    rj, rd = full_sort_reference(orc, R, S, 12)
    assert np.array_equal(j, rj)
    assert np.all(j[:, 9:] == -1) and np.all(np.isinf(dist[:, 9:]))
    assert all(sorted(j[i, :9].tolist()) == list(range(9)) for i in range(6))


def test_exclude_self(orc):
    X = synth.integer_grid_rows(40, 3, seed=4)
    j, d2, _ = orc.topk(X, None, 7, exclude_self=True)
    rj, rd = full_sort_reference(orc, X, X, 7, exclude_self=True)
    assert np.array_equal(j, rj)
    assert not np.any(j == np.arange(40)[:, None])
    rows = np.array([3, 9, 33])
    sj, _, _ = orc.topk(np.ascontiguousarray(X[rows]), X, 7, exclude_self=True, self_ids=rows)
    assert np.array_equal(sj, j[rows])


def test_topk_inside_eps_join_at_kth_distance(orc):
    R = synth.gaussian_mixture_unit(20, 8, 3, seed=5)
    S = synth.gaussian_mixture_unit(60, 8, 3, seed=5, stream=1)
    k = 6
    j, d2, dist = orc.topk(R, S, k)
    for i in range(20):
        eps = float(np.sqrt(d2[i, k - 1]))
        g = orc.eps_join(np.ascontiguousarray(R[i:i + 1]), S, eps)
        within = set(g["j"].tolist())
        assert set(j[i].tolist()) <= within
        # absent ties at the k-th distance, the two sets are equal
        if np.count_nonzero(orc.pair_d2(R, S, np.full(60, i), np.arange(60)) == d2[i, k - 1]) == 1:
            assert set(j[i].tolist()) == within
