"""CPU oracle for the patch-featurisation and similarity-join hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product path (``paper_1812_07607_amd``) never imports it and shares no code
with it.  The arithmetic lives in ``dl_oracle.c`` (plain C, fp64, sequential
per pair); this module only compiles it and marshals numpy arrays.

Paper: Krishnan et al., "DeepLens: Towards a Visual Data Management System"
(CIDR 2019).  Each wrapper names the passage its C function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: the canonical distance is a sequence of separately
# rounded double subtractions, multiplications and additions.
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
          "-shared", "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile ``dl_oracle.c`` into ``liboracle.so`` next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_hist_rgb8.argtypes = [P, i64, i32, i32, i32, P, P, i32]
        L.orc_hist_rgb8.restype = ctypes.c_int
        L.orc_hist_crops.argtypes = [P, i64, i32, i32, P, i64, i32, P, i32]
        L.orc_hist_crops.restype = ctypes.c_int
        L.orc_d2.argtypes = [P, P, i32]
        L.orc_d2.restype = f64
        L.orc_pair_d2.argtypes = [P, i64, P, i64, i32, P, P, i64, P, i32]
        L.orc_pair_d2.restype = None
        L.orc_eps_join.argtypes = [P, i64, i64, P, i64, i64, i32, f64, i32, P, i32,
                                   P, P, P, P, i64]
        L.orc_eps_join.restype = i64
        L.orc_topk.argtypes = [P, i64, i64, P, i64, i64, i32, i32, i32, P, i32, P, P, P]
        L.orc_topk.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32_rows(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x)
    if x.dtype != np.float32 or x.ndim != 2 or x.strides[1] != 4:
        raise TypeError("expected a 2-D float32 array with unit column stride")
    return x


def max_threads() -> int:
    return int(lib().orc_max_threads())


def hist_rgb8(patches: np.ndarray, bins: int = 8, nthreads: int = 0, counts: bool = False):
    """Colour histogram per patch (section "Visual ETL", Transformers).

    patches: (n, h, w, 3) uint8, R,G,B per pixel.  Returns (n, bins**3)
    float32 L1-normalised histograms, and the raw int32 counts if asked.
    """
    p = np.ascontiguousarray(patches, dtype=np.uint8)
    if p.ndim != 4 or p.shape[3] != 3:
        raise ValueError("patches must be (n, h, w, 3)")
    n, h, w, _ = p.shape
    nb = bins ** 3
    out = np.empty((n, nb), np.float32)
    cnt = np.empty((n, nb), np.int32) if counts else None
    rc = lib().orc_hist_rgb8(_ptr(p), n, h, w, bins, _ptr(out),
                             _ptr(cnt) if counts else None, nthreads)
    if rc != 0:
        raise ValueError("orc_hist_rgb8 failed with code %d" % rc)
    return (out, cnt) if counts else out


def hist_crops(frames: np.ndarray, boxes, bins: int = 8, nthreads: int = 0) -> np.ndarray:
    """Colour histograms of bounding boxes over frames (section "Iterator API
    for Patches": a patch is a region of an image; section "Visual ETL").

    frames: (nframes, height, width, 3) uint8; boxes: (m, 5) int (frame, x0,
    y0, x1, y1), pixels x0 <= x < x1, y0 <= y < y1.  Returns (m, bins**3)
    float32, each count divided by the box's pixel count.
    """
    f = np.ascontiguousarray(frames, dtype=np.uint8)
    if f.ndim != 4 or f.shape[3] != 3:
        raise ValueError("frames must be (nframes, height, width, 3)")
    bx = np.ascontiguousarray(boxes, dtype=np.int32).reshape(-1, 5)
    out = np.empty((bx.shape[0], bins ** 3), np.float32)
    rc = lib().orc_hist_crops(_ptr(f), f.shape[0], f.shape[1], f.shape[2], _ptr(bx), bx.shape[0], bins,
                              _ptr(out), nthreads)
    if rc != 0:
        raise ValueError("orc_hist_crops failed with code %d" % rc)
    return out


def d2(a: np.ndarray, b: np.ndarray) -> float:
    """Canonical squared L2 distance of two float32 vectors (fp64, sequential)."""
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    if a.shape != b.shape or a.ndim != 1:
        raise ValueError("vectors must be 1-D of equal length")
    return float(lib().orc_d2(_ptr(a), _ptr(b), a.shape[0]))


def pair_d2(R: np.ndarray, S: np.ndarray, pi, pj, nthreads: int = 0) -> np.ndarray:
    """Canonical d2 for the listed pairs (R[pi[t]], S[pj[t]])."""
    R, S = _f32_rows(R), _f32_rows(S)
    pi = np.ascontiguousarray(pi, np.int64)
    pj = np.ascontiguousarray(pj, np.int64)
    if pi.shape != pj.shape:
        raise ValueError("pi and pj differ in length")
    if len(pi) and (pi.min() < 0 or pi.max() >= R.shape[0] or pj.min() < 0 or pj.max() >= S.shape[0]):
        raise IndexError("pair index out of range")
    out = np.empty(len(pi), np.float64)
    lib().orc_pair_d2(_ptr(R), R.strides[0] // 4, _ptr(S), S.strides[0] // 4,
                      R.shape[1], _ptr(pi), _ptr(pj), len(pi), _ptr(out), nthreads)
    return out


def eps_join(R: np.ndarray, S: np.ndarray | None, eps: float, nthreads: int = 0,
             cap: int | None = None, self_join: bool | None = None, row_ids=None):
    """Nested-loop eps-join (section "Query Processing", Nested Loop Join).

    S=None means the self-join of R with i < j.  For a sample of rows of a
    self-join pass R = the sampled rows, S = the full relation,
    self_join=True and row_ids = their (increasing) indices in S.  Returns a
    dict with int64 arrays i, j, fp64 d2, float32 dist, in (i, j) order, and
    the total count.
    """
    if self_join is None:
        self_join = S is None
    R = _f32_rows(R)
    S = R if S is None else _f32_rows(S)
    if R.shape[1] != S.shape[1]:
        raise ValueError("R and S differ in dimension")
    rid = None
    if row_ids is not None:
        rid = np.ascontiguousarray(row_ids, np.int64)
        if rid.shape != (R.shape[0],):
            raise ValueError("row_ids must give one index per row of R")
    L = lib()
    args = (_ptr(R), R.shape[0], R.strides[0] // 4, _ptr(S), S.shape[0],
            S.strides[0] // 4, R.shape[1], float(eps), int(self_join),
            _ptr(rid) if rid is not None else None, nthreads)
    if cap is None:
        total = L.orc_eps_join(*args, None, None, None, None, 0)
        if total < 0:
            raise ValueError("orc_eps_join failed with code %d" % -total)
        cap = total
    oi = np.empty(cap, np.int64)
    oj = np.empty(cap, np.int64)
    od = np.empty(cap, np.float64)
    odist = np.empty(cap, np.float32)
    total = L.orc_eps_join(*args, _ptr(oi), _ptr(oj), _ptr(od), _ptr(odist), cap)
    if total < 0:
        raise ValueError("orc_eps_join failed with code %d" % -total)
    m = min(cap, total)
    return {"i": oi[:m], "j": oj[:m], "d2": od[:m], "dist": odist[:m], "count": int(total)}


def topk(R: np.ndarray, S: np.ndarray | None, k: int, exclude_self: bool = False,
         nthreads: int = 0, self_ids=None):
    """Top-k closest entries of S per row of R (query q1, section "Queries").

    S=None means S is R.  self_ids (optional) gives the index in S of each row
    of R, for excluding the row itself when R is a sample of S.  Returns
    (j int64 (nR,k), d2 fp64, dist float32); padding is j = -1,
    d2 = dist = +inf.
    """
    R = _f32_rows(R)
    sid = None
    if self_ids is not None:
        sid = np.ascontiguousarray(self_ids, np.int64)
        if sid.shape != (R.shape[0],):
            raise ValueError("self_ids must give one index per row of R")
    S = R if S is None else _f32_rows(S)
    if R.shape[1] != S.shape[1]:
        raise ValueError("R and S differ in dimension")
    nR = R.shape[0]
    oj = np.empty((nR, k), np.int64)
    od = np.empty((nR, k), np.float64)
    odist = np.empty((nR, k), np.float32)
    rc = lib().orc_topk(_ptr(R), nR, R.strides[0] // 4, _ptr(S), S.shape[0],
                        S.strides[0] // 4, R.shape[1], k, int(exclude_self),
                        _ptr(sid) if sid is not None else None,
                        nthreads, _ptr(oj), _ptr(od), _ptr(odist))
    if rc != 0:
        raise ValueError("orc_topk failed with code %d" % rc)
    return oj, od, odist
