"""Pins for the oracle's distance and eps-join.

Passages: section "Query Processing" (Nested Loop Join: compare all pairs,
keep those meeting the predicate) and section "Derived Data" (Euclidean
threshold queries on image features).  Checked against hand-computed values,
exact rational arithmetic on tiny inputs, closed forms and invariants."""
import math
from fractions import Fraction

import numpy as np
import pytest

from conftest import read_golden
from paper_1812_07607_amd import synth


def exact_d2(a, b):
    """Exact squared distance of two float32 vectors as a Fraction."""
    return sum((Fraction(float(x)) - Fraction(float(y))) ** 2 for x, y in zip(a, b))


def gamma(n, u=2.0 ** -53):
    return n * u / (1 - n * u)


def test_hand_eps_join(orc):
    rows = read_golden("eps_join_hand.txt")
    R = np.array([list(map(float, r[1:])) for r in rows if r[0] == "R"], np.float32)
    S = np.array([list(map(float, r[1:])) for r in rows if r[0] == "S"], np.float32)
    eps = float([r for r in rows if r[0] == "eps"][0][1])
    expect = [(int(r[1]), int(r[2]), float(r[3])) for r in rows if r[0] == "pair"]
    got = orc.eps_join(R, S, eps)
    assert got["count"] == len(expect)
    assert list(zip(got["i"].tolist(), got["j"].tolist(), got["dist"].tolist())) == expect


def test_pythagorean_closed_form(orc):
    # (3/8, 4/8) against the origin: d2 = 25/64 and dist = 5/8 exactly
    a = np.array([3 / 8, 4 / 8], np.float32)
    z = np.zeros(2, np.float32)
    assert orc.d2(a, z) == 25 / 64
    # scaled Pythagorean quadruple (1, 2, 2) / 16: d = 3/16
    b = np.array([1 / 16, 2 / 16, 2 / 16, 0.0], np.float32)
    assert orc.d2(b, np.zeros(4, np.float32)) == (3 / 16) ** 2


def test_identity_and_bitwise_symmetry(orc):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((30, 33)).astype(np.float32)
    for i in range(30):
        assert orc.d2(X[i], X[i]) == 0.0
        for j in range(30):
            assert orc.d2(X[i], X[j]) == orc.d2(X[j], X[i])


@pytest.mark.parametrize("d", [1, 3, 8])
def test_d2_within_rounding_of_exact(orc, d):
    rng = np.random.default_rng(d)
    X = (rng.standard_normal((12, d)) * rng.choice([1e-3, 1.0, 1e3], size=(12, 1))).astype(np.float32)
    for i in range(12):
        for j in range(12):
            ex = exact_d2(X[i], X[j])
            got = Fraction(orc.d2(X[i], X[j]))
            # each difference, square and add rounds once in double
            assert abs(got - ex) <= Fraction(gamma(d + 2)) * ex


def read_d2_order_cases():
    """Cases of tests/golden/d2_order.txt: name -> (a, b, expected d2)."""
    cases, cur = {}, None
    for row in read_golden("d2_order.txt"):
        if row[0] == "case":
            cur = row[1]
            cases[cur] = {}
        elif row[0] in ("a", "b"):
            cases[cur][row[0]] = np.array([float.fromhex(v) for v in row[1:]], np.float32)
        elif row[0] == "d2":
            cases[cur]["d2"] = float.fromhex(row[1])
    return {k: (v["a"], v["b"], v["d2"]) for k, v in cases.items()}


@pytest.mark.parametrize("case", ["order", "fma"])
def test_canonical_summation_order_golden(orc, case):
    """The float64 value follows the canonical sequence bit for bit: summed
    in increasing k, each operation rounded on its own (hand-worked values;
    reversing the loop changes the 'order' case, a fused multiply-add the
    'fma' case)."""
    a, b, expect = read_d2_order_cases()[case]
    got = orc.d2(a, b)
    assert got == expect, "%s: %s vs %s" % (case, got.hex(), expect.hex())
    # the eps-join and top-k report the same canonical value
    R, S = a[None, :].copy(), b[None, :].copy()
    assert orc.eps_join(R, S, math.inf)["d2"][0] == expect
    assert orc.topk(R, S, 1)[1][0, 0] == expect


def test_integer_grid_is_exact(orc):
    # vectors with small dyadic entries: every operation is exact in double
    rng = np.random.default_rng(5)
    X = (rng.integers(-64, 65, size=(20, 16)) / 64.0).astype(np.float32)
    for i in range(20):
        for j in range(20):
            assert Fraction(orc.d2(X[i], X[j])) == exact_d2(X[i], X[j])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_eps_join_matches_exact_rational_brute_force(orc, seed):
    rng = np.random.default_rng(seed)
    n, m, d = 25, 31, 6
    R = rng.standard_normal((n, d)).astype(np.float32)
    S = rng.standard_normal((m, d)).astype(np.float32)
    S[:3] = R[:3]  # planted duplicates
    ex = {(i, j): exact_d2(R[i], S[j]) for i in range(n) for j in range(m)}
    vals = sorted(ex.values())
    near_boundary = 0
    for eps in [0.0, float(math.sqrt(vals[len(vals) // 10])), 1.5, 1e9]:
        got = orc.eps_join(R, S, eps)
        got_set = set(zip(got["i"].tolist(), got["j"].tolist()))
        e2 = Fraction(eps) ** 2
        for (i, j), v in ex.items():
            inside = v <= e2
            if abs(v - e2) <= Fraction(gamma(d + 4)) * max(v, e2):
                near_boundary += 1  # rounding may decide these; sqrt-predicate governs
                continue
            assert ((i, j) in got_set) == inside, (i, j, eps)
    # the order statistic used as eps is itself a d2 value, so its own pair
    # is at the boundary: the inclusive predicate must keep it
    eps = float(np.sqrt(float(vals[len(vals) // 10])))
    got = orc.eps_join(R, S, eps)
    assert got["count"] >= 1


def test_eps_extremes_and_monotone(orc):
    rng = np.random.default_rng(9)
    R = rng.standard_normal((40, 5)).astype(np.float32)
    S = rng.standard_normal((35, 5)).astype(np.float32)
    S[7] = R[4]
    S[20] = R[4]
    assert orc.eps_join(R, S, math.inf)["count"] == 40 * 35
    z = orc.eps_join(R, S, 0.0)
    assert list(zip(z["i"].tolist(), z["j"].tolist())) == [(4, 7), (4, 20)]
    prev = None
    for eps in np.linspace(0, 6, 25):
        cur = set(zip(*[a.tolist() for a in (lambda g: (g["i"], g["j"]))(orc.eps_join(R, S, eps))]))
        if prev is not None:
            assert prev <= cur
        prev = cur


def test_self_join_is_upper_half_of_symmetric_full_join(orc):
    R = synth.dirichlet_clusters(60, 16, 4, seed=1)
    R[10] = R[3]
    eps = 0.15
    full = orc.eps_join(R, R.copy(), eps)
    fs = set(zip(full["i"].tolist(), full["j"].tolist()))
    assert all((j, i) in fs for (i, j) in fs)  # symmetric
    self_j = orc.eps_join(R, None, eps)
    ss = list(zip(self_j["i"].tolist(), self_j["j"].tolist()))
    assert ss == sorted(p for p in fs if p[0] < p[1])
    assert (3, 10) in ss


def test_output_order_and_distances(orc):
    R = synth.dirichlet_clusters(50, 8, 3, seed=2)
    S = synth.dirichlet_clusters(70, 8, 3, seed=2, stream=1)
    g = orc.eps_join(R, S, 0.2)
    keys = list(zip(g["i"].tolist(), g["j"].tolist()))
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    for i, j, d2, dist in zip(g["i"], g["j"], g["d2"], g["dist"]):
        assert d2 == orc.d2(R[i], S[j])
        assert dist == np.float32(np.sqrt(d2))


def test_cap_returns_first_entries(orc):
    R = synth.dirichlet_clusters(30, 8, 2, seed=4)
    full = orc.eps_join(R, None, 0.5)
    part = orc.eps_join(R, None, 0.5, cap=7)
    assert part["count"] == full["count"] and len(part["i"]) == min(7, full["count"])
    assert np.array_equal(part["i"], full["i"][:7]) and np.array_equal(part["j"], full["j"][:7])


def test_sampled_rows_equal_subset_of_full(orc):
    X = synth.dirichlet_clusters(80, 8, 3, seed=6)
    full = orc.eps_join(X, None, 0.3)
    rows = np.array([0, 5, 17, 40, 79])
    sub = orc.eps_join(np.ascontiguousarray(X[rows]), X, 0.3, self_join=True, row_ids=rows)
    sel = np.isin(full["i"], rows)
    assert np.array_equal(sub["i"], full["i"][sel]) and np.array_equal(sub["j"], full["j"][sel])
    assert np.array_equal(sub["d2"], full["d2"][sel])


def test_histogram_integer_identity(orc):
    """For L1-normalised histograms of 1024-pixel patches every entry is
    count/2^10, so d2 * 2^20 equals the integer sum of squared count
    differences; the counts come from numpy.histogramdd, not the oracle."""
    from test_oracle_hist import histogramdd_reference
    patches, _ = synth.patches_palette(24, 32, 32, 4, 20.0, seed=8)
    H = orc.hist_rgb8(patches, 8)
    C = histogramdd_reference(patches, 8)
    for i in range(24):
        for j in range(24):
            diff = C[i] - C[j]
            assert orc.d2(H[i], H[j]) * 2 ** 20 == float(np.dot(diff, diff))


def test_pair_d2_matches_d2(orc):
    R = synth.uniform_rows(20, 9, seed=1)
    S = synth.uniform_rows(15, 9, seed=1, stream=1)
    pi, pj = synth.sample_pairs(20, 15, 50, False, 3)
    v = orc.pair_d2(R, S, pi, pj)
    assert all(v[t] == orc.d2(R[pi[t]], S[pj[t]]) for t in range(50))
