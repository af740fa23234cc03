"""Helpers for the GPU parity tests: device transfer and the comparison rules.

Pair and index sets must equal the oracle's bit for bit.  Distances are
float32: for pairs decided in float32 the error of d2_32 against the
canonical d2_64 is at most 2 gamma_{d+2} d2 (+ tiny absolute terms), so the
distance is within (d+2) 2^-24 relative plus one float32 rounding; pairs on a
dyadic grid are exact."""
import numpy as np
import torch


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def dist_tol(d):
    return (d + 2) * 2.0 ** -24 * 1.01 + 2.0 ** -23


def assert_dist_close(got, ref, d, what=""):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin), what
    err = np.abs(got[fin] - ref[fin])
    lim = ref[fin] * dist_tol(d) + 1e-37
    bad = err > lim
    assert not bad.any(), "%s: %d distances off, worst rel %.3g" % (what, bad.sum(), (err / np.maximum(ref[fin], 1e-300)).max())


def assert_eps_equal(gpu, ref, d, what=""):
    """gpu: ops.EpsResult; ref: oracle.eps_join dict."""
    assert gpu.count == ref["count"], "%s: count %d vs oracle %d" % (what, gpu.count, ref["count"])
    gi = host(gpu.i).astype(np.int64) & 0xffffffff
    gj = host(gpu.j).astype(np.int64) & 0xffffffff
    assert np.array_equal(gi, ref["i"]), what + ": i differs"
    assert np.array_equal(gj, ref["j"]), what + ": j differs"
    assert_dist_close(host(gpu.dist), ref["dist"], d, what)


def assert_topk_equal(gpu, ref_j, ref_dist, d, what=""):
    gj = host(gpu.j).astype(np.int64)
    gj[gj < 0] = -1
    bad = np.nonzero((gj != ref_j).any(axis=1))[0]
    assert len(bad) == 0, "%s: %d rows differ, first row %d: gpu %s oracle %s" % (
        what, len(bad), bad[0], gj[bad[0]].tolist(), ref_j[bad[0]].tolist())
    assert_dist_close(host(gpu.dist), ref_dist, d, what)
