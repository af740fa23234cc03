"""The no-allocation eps-join (dl_join_eps_noalloc) against dl_join_eps.

Both are called through the C ABI on the same inputs; the pair arrays must
be equal bit for bit and in order, and equal to the float64 oracle's.  Two
calls in a row, the second smaller, so the fixed scratch carries the first
call's contents into the second."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import assert_dist_close, dev, host
from paper_1812_07607_amd import _lib, ops, synth

pytestmark = pytest.mark.gpu


def _pairs(cap, device):
    oi = torch.full((cap,), -7, dtype=torch.int32, device=device)
    oj = torch.full((cap,), -7, dtype=torch.int32, device=device)
    od = torch.full((cap,), float("nan"), dtype=torch.float32, device=device)
    pr = _lib.dl_pairs(oi.data_ptr(), oj.data_ptr(), od.data_ptr(), cap, 0, 0, 0)
    return (oi, oj, od), pr


def _call_both(R, S, eps, prec, cap):
    c = ops.context()
    L = c.L
    self_join = S is None
    Rt = dev(R)
    St = Rt if self_join else dev(S)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # the existing entry point, with a workspace from torch
    need = L.dl_join_eps_workspace(Rt.shape[0], St.shape[0], Rt.shape[1], _lib.PREC[prec], int(self_join), 1 << 20)
    ws = torch.empty(int(need), dtype=torch.uint8, device=Rt.device)
    a, pa = _pairs(cap, Rt.device)
    st = L.dl_join_eps(c.h, ops._mat(Rt), ops._mat(St), int(self_join), float(eps), _lib.PREC[prec],
                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(pa), stream)
    assert st == _lib.DL_OK, L.dl_last_error(c.h)
    # the no-allocation entry point
    b, pb = _pairs(cap, Rt.device)
    st = L.dl_join_eps_noalloc(c.h, ops._mat(Rt), ops._mat(St), int(self_join), float(eps), _lib.PREC[prec],
                               ctypes.byref(pb), stream)
    assert st == _lib.DL_OK, L.dl_last_error(c.h)
    return (a, pa), (b, pb)


def _check(orc, R, S, eps, prec, d):
    cap = 1 << 16
    (a, pa), (b, pb) = _call_both(R, S, eps, prec, cap)
    assert pb.count == pa.count and pb.candidates == pa.candidates and pb.ties == pa.ties
    m = int(pa.count)
    assert 0 < m <= cap
    for x, y in zip(a, b):
        assert torch.equal(x[:m], y[:m])
    ref = orc.eps_join(R, S, eps)
    assert m == ref["count"]
    gi = host(b[0][:m]).astype(np.int64) & 0xffffffff
    gj = host(b[1][:m]).astype(np.int64) & 0xffffffff
    assert np.array_equal(gi, ref["i"]) and np.array_equal(gj, ref["j"])
    assert_dist_close(host(b[2][:m]), ref["dist"], d, "noalloc/" + prec)
    return m


def _eps(orc, R, S, q, seed):
    nS = R.shape[0] if S is None else S.shape[0]
    pi, pj = synth.sample_pairs(R.shape[0], nS, 4000, S is None, seed=seed)
    d2 = orc.pair_d2(R, R if S is None else S, pi, pj)
    return float(np.sqrt(synth.order_statistic(d2, q)))


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp8"])
def test_noalloc_matches_workspace_call_twice(orc, prec):
    # first call: 2,000 x 3,000 at d = 64; second: a smaller ragged self-join
    R1 = synth.gaussian_mixture_unit(2000, 64, 12, seed=71)
    S1 = synth.gaussian_mixture_unit(3000, 64, 12, seed=71, stream=1)
    m1 = _check(orc, R1, S1, _eps(orc, R1, S1, 0.01, 3), prec, 64)
    R2 = synth.gaussian_mixture_unit(517, 40, 5, seed=72)
    R2[300] = R2[17]  # a planted duplicate
    m2 = _check(orc, R2, None, _eps(orc, R2, None, 0.02, 4), prec, 40)
    assert m1 > 0 and m2 > 0


def test_noalloc_rejects_joins_beyond_the_scratch():
    c = ops.context()
    L = c.L
    # 12,000 x 12,000 at d = 1024 in fp32: the two operand copies alone exceed 64 MiB
    n, d = 12000, 1024
    need = L.dl_join_eps_workspace(n, n, d, _lib.PREC["fp32"], 0, 1)
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    x = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    y = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    _, pr = _pairs(16, x.device)
    st = L.dl_join_eps_noalloc(c.h, ops._mat(x), ops._mat(y), 0, 0.5, _lib.PREC["fp32"], ctypes.byref(pr),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.DL_ERR_WORKSPACE
    assert b"fixed scratch" in L.dl_last_error(c.h)
    assert L.dl_required_workspace(c.h) == 0
