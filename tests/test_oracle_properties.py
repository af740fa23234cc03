"""Property tests of the oracle (hypothesis): on random small relations of
dyadic values (multiples of 1/64 below 2 in magnitude, so every squared
distance is exact in float64), the eps-join is exactly the set of pairs
whose correctly rounded distance is at most eps -- eps drawn from the
pairs' own distances as often as not, so boundary pairs are common -- in
(i, j) order, the self-join its i < j half, and the top-k the k smallest
(d2, j) per row.  The reference side is written with exact integers and
math.sqrt (correctly rounded), independently of the oracle's C code."""
import math

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

DYADIC = st.integers(min_value=-127, max_value=127)


@st.composite
def relations(draw):
    d = draw(st.integers(1, 5))
    n = draw(st.integers(1, 7))
    m = draw(st.integers(1, 7))
    R = np.array(draw(st.lists(st.lists(DYADIC, min_size=d, max_size=d), min_size=n, max_size=n)), np.int64)
    S = np.array(draw(st.lists(st.lists(DYADIC, min_size=d, max_size=d), min_size=m, max_size=m)), np.int64)
    if draw(st.booleans()):  # a planted duplicate
        S[draw(st.integers(0, m - 1))] = R[draw(st.integers(0, n - 1))]
    return R, S


def d2_exact(a, b):
    """Squared distance of two rows of integers k (values k / 64), exact."""
    return int(((a - b) ** 2).sum()) / 4096.0  # an integer below 2^20 over 2^12: exact in float64


def ref_eps(R, S, eps, self_join):
    out = []
    for i in range(len(R)):
        for j in range(i + 1 if self_join else 0, len(S)):
            if math.sqrt(d2_exact(R[i], S[j])) <= eps:
                out.append((i, j))
    return out


def pick_eps(draw, R, S):
    choice = draw(st.integers(0, 3))
    if choice == 0:
        return 0.0
    if choice == 1:
        return float(draw(st.floats(min_value=0.0, max_value=8.0, allow_nan=False)))
    i = draw(st.integers(0, len(R) - 1))
    j = draw(st.integers(0, len(S) - 1))
    e = math.sqrt(d2_exact(R[i], S[j]))  # a pair exactly on the boundary
    return e if choice == 2 else math.nextafter(e, 0.0)


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(data=st.data())
def test_eps_join_is_the_rounded_distance_predicate(orc, data):
    R, S = data.draw(relations())
    eps = pick_eps(data.draw, R, S)
    Rf, Sf = (R / 64.0).astype(np.float32), (S / 64.0).astype(np.float32)
    got = orc.eps_join(Rf, Sf, eps)
    assert list(zip(got["i"].tolist(), got["j"].tolist())) == ref_eps(R, S, eps, False)
    for t in range(got["count"]):
        v = d2_exact(R[got["i"][t]], S[got["j"][t]])
        assert got["d2"][t] == v and got["dist"][t] == np.float32(math.sqrt(v))
    got = orc.eps_join(Rf, None, eps)
    assert list(zip(got["i"].tolist(), got["j"].tolist())) == ref_eps(R, R, eps, True)


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(data=st.data())
def test_topk_is_the_k_smallest_d2_then_j(orc, data):
    R, S = data.draw(relations())
    self_join = data.draw(st.booleans())
    if self_join:
        S = R
    k = data.draw(st.integers(1, len(S) + 2))
    excl = self_join and data.draw(st.booleans())
    Rf, Sf = (R / 64.0).astype(np.float32), (S / 64.0).astype(np.float32)
    j, d2, dist = orc.topk(Rf, None if self_join else Sf, k, exclude_self=excl)
    for i in range(len(R)):
        cand = sorted((d2_exact(R[i], S[c]), c) for c in range(len(S)) if not (excl and c == i))[:k]
        pad = k - len(cand)
        assert j[i].tolist() == [c for _, c in cand] + [-1] * pad, i
        assert d2[i].tolist() == [v for v, _ in cand] + [math.inf] * pad, i
        assert dist[i].tolist() == [float(np.float32(math.sqrt(v))) for v, _ in cand] + [math.inf] * pad, i
