"""Python entry points over libdlmi.so, on torch device tensors.

PyTorch supplies device memory (tensors) and streams; every step of the
featurisation and the joins runs in the library's HIP kernels.  Calls go to
the GPU path only: when the library or a GPU is missing they raise.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib

_ctx_cache = {}


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """One dl_ctx per device (created lazily, destroyed at exit)."""

    def __init__(self, device: int = 0):
        L = _lib.load()
        self.L = L
        self.device = device
        h = ctypes.c_void_p()
        st = L.dl_create(device, ctypes.byref(h))
        if st != _lib.DL_OK:
            raise _lib.DLError(st, "dl_create(%d) failed" % device)
        self.h = h
        self.band_caps = {}  # top-k call shape -> band capacity that sufficed
        self.eps_caps = {}   # eps-join call shape and eps -> output capacity that sufficed

    def check(self, st: int):
        if st != _lib.DL_OK:
            raise _lib.DLError(st, self.L.dl_last_error(self.h).decode())

    def band_full(self, st: int) -> bool:
        """A top-k call failed only because a row's band buffer was full (a
        larger band_cap helps; more near-tie contenders than the selection
        holds does not)."""
        return st == _lib.DL_ERR_WORKSPACE and b"band buffer" in (self.L.dl_last_error(self.h) or b"")

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.L.dl_destroy(self.h)
        except Exception:
            pass

    def set_timing(self, on: bool):
        self.check(self.L.dl_set_timing(self.h, int(on)))

    def timing(self, reset: bool = False):
        ms = (ctypes.c_double * _lib.NUM_STAGES)()
        calls = (ctypes.c_int64 * _lib.NUM_STAGES)()
        self.check(self.L.dl_get_timing(self.h, ms, calls, int(reset)))
        return {name: (ms[s], calls[s]) for s, name in enumerate(_lib.STAGES)}


def context(device=None) -> Context:
    if not torch.cuda.is_available():
        raise RuntimeError("the dlmi library needs a ROCm GPU; none is visible")
    dev = torch.cuda.current_device() if device is None else int(device)
    c = _ctx_cache.get(dev)
    if c is None:
        c = _ctx_cache[dev] = Context(dev)
    return c


def _mat(x: torch.Tensor) -> _lib.dl_mat:
    if x.dtype != torch.float32 or x.dim() != 2 or not x.is_cuda:
        raise TypeError("expected a 2-D float32 CUDA tensor")
    if x.shape[0] > 0 and x.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    ld = x.stride(0) if x.shape[0] > 1 else x.shape[1]
    return _lib.dl_mat(x.data_ptr(), x.shape[0], x.shape[1], max(ld, x.shape[1]))


# ---------------------------------------------------------------- featurise
def featurize_rgb8(patches: torch.Tensor, bins: int = 8, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """Colour histograms (bins^3, L1-normalised) of uint8 (n, h, w, 3) patches."""
    if patches.dtype != torch.uint8 or patches.dim() != 4 or patches.shape[3] != 3 or not patches.is_cuda:
        raise TypeError("patches must be a (n, h, w, 3) uint8 CUDA tensor")
    patches = patches.contiguous()
    n, h, w, _ = patches.shape
    if out is None:
        out = torch.empty((n, bins ** 3), dtype=torch.float32, device=patches.device)
    c = context(patches.device.index)
    c.check(c.L.dl_featurize_rgb8(c.h, ctypes.c_void_p(patches.data_ptr()), n, h, w, bins,
                                  ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def featurize_crops_rgb8(frames: torch.Tensor, boxes: torch.Tensor, bins: int = 8, out: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
    """Colour histograms of boxes (int32 (m, 5): frame, x0, y0, x1, y1) over
    uint8 (nframes, height, width, 3) frames."""
    if frames.dtype != torch.uint8 or frames.dim() != 4 or frames.shape[3] != 3 or not frames.is_cuda:
        raise TypeError("frames must be a (nframes, height, width, 3) uint8 CUDA tensor")
    frames = frames.contiguous()
    boxes = boxes.to(device=frames.device, dtype=torch.int32).contiguous().reshape(-1, 5)
    nf, hh, ww, _ = frames.shape
    m = boxes.shape[0]
    if out is None:
        out = torch.empty((m, bins ** 3), dtype=torch.float32, device=frames.device)
    c = context(frames.device.index)
    c.check(c.L.dl_featurize_crops_rgb8(c.h, ctypes.c_void_p(frames.data_ptr()), nf, hh, ww,
                                        ctypes.c_void_p(boxes.data_ptr()), m, bins, ctypes.c_void_p(out.data_ptr()),
                                        _stream_ptr(stream)))
    return out


# ---------------------------------------------------------------- distances
def pair_d2(R: torch.Tensor, S: torch.Tensor, pi: torch.Tensor, pj: torch.Tensor, stream=None) -> torch.Tensor:
    """Canonical float64 squared distances of listed pairs."""
    pi = pi.to(device=R.device, dtype=torch.int32).contiguous()
    pj = pj.to(device=R.device, dtype=torch.int32).contiguous()
    out = torch.empty(pi.shape[0], dtype=torch.float64, device=R.device)
    c = context(R.device.index)
    c.check(c.L.dl_pair_d2(c.h, _mat(R), _mat(S), ctypes.c_void_p(pi.data_ptr()), ctypes.c_void_p(pj.data_ptr()),
                           pi.shape[0], ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


# ---------------------------------------------------------------- eps-join
@dataclass
class EpsResult:
    i: torch.Tensor      # int32 (as uint32 bits), sorted by (i, j)
    j: torch.Tensor
    dist: torch.Tensor   # float32
    count: int
    candidates: int
    ties: int


class Workspace:
    """Growable device scratch buffer (a torch uint8 tensor)."""

    def __init__(self, device):
        self.device = device
        self.buf = torch.empty(0, dtype=torch.uint8, device=device)

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        return self.buf


_ws = {}


def _workspace(device) -> Workspace:
    w = _ws.get(device)
    if w is None:
        w = _ws[device] = Workspace(device)
    return w


def join_eps(R: torch.Tensor, S: torch.Tensor | None, eps: float, prec: str = "bf16",
             max_candidates: int | None = None, capacity: int | None = None, stream=None,
             workspace: Workspace | None = None, out: tuple | None = None) -> EpsResult:
    """eps-join: all (i, j) with canonical distance <= eps (S=None: self-join
    of R with i < j), sorted by (i, j).  Grows the workspace and the output
    and retries when either is too small."""
    self_join = S is None
    Sm = R if self_join else S
    c = context(R.device.index)
    ws = workspace or _workspace(R.device)
    p = _lib.PREC[prec]
    nR, nS, d = R.shape[0], Sm.shape[0], R.shape[1]
    if max_candidates is None:
        max_candidates = max(1 << 20, 4 * (nR + nS))
    cap = capacity if capacity is not None else max(1 << 16, nR + nS)
    # a call of the same shape and eps starts from the output size that
    # sufficed last time instead of failing on capacity again
    key = (nR, nS, d, p, self_join, float(eps))
    if capacity is None:
        cap = max(cap, c.eps_caps.get(key, 0))
    if out is not None and capacity is None:
        cap = out[0].numel()
    for _ in range(8):
        need = c.L.dl_join_eps_workspace(nR, nS, d, p, int(self_join), max_candidates)
        buf = ws.get(need)
        if out is not None and out[0].numel() >= cap:
            oi, oj, od = out
        else:
            oi = torch.empty(cap, dtype=torch.int32, device=R.device)
            oj = torch.empty(cap, dtype=torch.int32, device=R.device)
            od = torch.empty(cap, dtype=torch.float32, device=R.device)
        pr = _lib.dl_pairs(oi.data_ptr(), oj.data_ptr(), od.data_ptr(), cap, 0, 0, 0)
        st = c.L.dl_join_eps(c.h, _mat(R), _mat(Sm), int(self_join), float(eps), p,
                             ctypes.c_void_p(buf.data_ptr()), buf.numel(), ctypes.byref(pr), _stream_ptr(stream))
        if st == _lib.DL_ERR_WORKSPACE:
            req = c.L.dl_required_workspace(c.h)
            max_candidates = max(2 * max_candidates, int(pr.candidates * 1.25) + 1024)
            if req > 0 and c.L.dl_join_eps_workspace(nR, nS, d, p, int(self_join), max_candidates) < req:
                max_candidates *= 2
            continue
        if st == _lib.DL_ERR_CAPACITY:
            cap = int(pr.count)
            out = None
            continue
        c.check(st)
        m = int(pr.count)
        if capacity is None:
            c.eps_caps[key] = cap
        return EpsResult(oi[:m], oj[:m], od[:m], m, int(pr.candidates), int(pr.ties))
    raise RuntimeError("join_eps did not converge on workspace / capacity")


@dataclass
class IndexInfo:
    tiles_total: int     # 256 x 256 tiles of the join (self-join: upper triangle)
    tiles_computed: int  # tiles the candidate pass ran on
    pivots: int          # 0: no index was built (the plain join ran)
    ksteps_per_tile: int = 0  # K-steps (128 operand bytes per row) of a full tile
    ksteps_computed: int = 0  # K-steps run: steps zero in every row of either tile are skipped


def join_eps_indexed(R: torch.Tensor, S: torch.Tensor | None, eps: float, prec: str = "bf16", pivots: int = 0,
                     max_candidates: int | None = None, capacity: int | None = None, stream=None,
                     workspace: Workspace | None = None):
    """eps-join with an index built on the fly (block balls over rows ordered
    by nearest pivot; tiles that cannot hold a result pair are skipped).  Same
    result as join_eps; returns (EpsResult, IndexInfo)."""
    self_join = S is None
    Sm = R if self_join else S
    c = context(R.device.index)
    ws = workspace or _workspace(R.device)
    p = _lib.PREC[prec]
    nR, nS, d = R.shape[0], Sm.shape[0], R.shape[1]
    if max_candidates is None:
        max_candidates = max(1 << 20, 4 * (nR + nS))
    cap = capacity if capacity is not None else max(1 << 16, nR + nS)
    key = ("indexed", nR, nS, d, p, self_join, float(eps), int(pivots))
    if capacity is None:
        cap = max(cap, c.eps_caps.get(key, 0))
    info = _lib.dl_index_info()
    for _ in range(8):
        need = c.L.dl_join_eps_indexed_workspace(nR, nS, d, p, int(self_join), max_candidates, pivots)
        buf = ws.get(need)
        oi = torch.empty(cap, dtype=torch.int32, device=R.device)
        oj = torch.empty(cap, dtype=torch.int32, device=R.device)
        od = torch.empty(cap, dtype=torch.float32, device=R.device)
        pr = _lib.dl_pairs(oi.data_ptr(), oj.data_ptr(), od.data_ptr(), cap, 0, 0, 0)
        st = c.L.dl_join_eps_indexed(c.h, _mat(R), _mat(Sm), int(self_join), float(eps), p, int(pivots),
                                     ctypes.c_void_p(buf.data_ptr()), buf.numel(), ctypes.byref(pr),
                                     ctypes.byref(info), _stream_ptr(stream))
        if st == _lib.DL_ERR_WORKSPACE:
            max_candidates = max(2 * max_candidates, int(pr.candidates * 1.25) + 1024)
            continue
        if st == _lib.DL_ERR_CAPACITY:
            cap = int(pr.count)
            continue
        c.check(st)
        m = int(pr.count)
        if capacity is None:
            c.eps_caps[key] = cap
        return (EpsResult(oi[:m], oj[:m], od[:m], m, int(pr.candidates), int(pr.ties)),
                IndexInfo(int(info.tiles_total), int(info.tiles_computed), int(info.pivots),
                          int(info.ksteps_per_tile), int(info.ksteps_computed)))
    raise RuntimeError("join_eps_indexed did not converge on workspace / capacity")


def join_eps_filtered(R: torch.Tensor, S: torch.Tensor | None, eps: float, labels_R: torch.Tensor,
                      labels_S: torch.Tensor | None, label: int, plan: str = "filter_first", prec: str = "bf16",
                      max_candidates: int | None = None, max_pairs: int | None = None, capacity: int | None = None,
                      stream=None, workspace: Workspace | None = None) -> EpsResult:
    """eps-join of the rows whose int32 label equals `label`, with the label
    filter before the match (plan "filter_first") or after it
    ("match_first").  The same result either way."""
    self_join = S is None
    Sm = R if self_join else S
    lR = labels_R.to(device=R.device, dtype=torch.int32).contiguous()
    lS = lR if self_join else labels_S.to(device=R.device, dtype=torch.int32).contiguous()
    c = context(R.device.index)
    ws = workspace or _workspace(R.device)
    p = _lib.PREC[prec]
    pl = {"filter_first": 0, "match_first": 1}[plan]
    nR, nS, d = R.shape[0], Sm.shape[0], R.shape[1]
    if max_candidates is None:
        max_candidates = max(1 << 20, 4 * (nR + nS))
    if max_pairs is None:
        max_pairs = max(1 << 20, 4 * (nR + nS))
    cap = capacity if capacity is not None else max(1 << 16, nR + nS)
    key = ("filtered", nR, nS, d, p, self_join, float(eps), int(label), pl)
    if capacity is None:
        cap = max(cap, c.eps_caps.get(key, 0))
    for _ in range(10):
        need = c.L.dl_join_eps_filtered_workspace(nR, nS, d, p, int(self_join), pl, max_candidates, max_pairs)
        buf = ws.get(need)
        oi = torch.empty(cap, dtype=torch.int32, device=R.device)
        oj = torch.empty(cap, dtype=torch.int32, device=R.device)
        od = torch.empty(cap, dtype=torch.float32, device=R.device)
        pr = _lib.dl_pairs(oi.data_ptr(), oj.data_ptr(), od.data_ptr(), cap, 0, 0, 0)
        st = c.L.dl_join_eps_filtered(c.h, _mat(R), _mat(Sm), int(self_join), float(eps), p,
                                      ctypes.c_void_p(lR.data_ptr()), ctypes.c_void_p(lS.data_ptr()), int(label), pl,
                                      max_candidates, max_pairs, ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                      ctypes.byref(pr), _stream_ptr(stream))
        if st == _lib.DL_ERR_WORKSPACE:
            max_candidates = max(2 * max_candidates, int(pr.candidates * 1.25) + 1024)
            max_pairs = max(2 * max_pairs, int(pr.count * 1.25) + 1024)
            continue
        if st == _lib.DL_ERR_CAPACITY:
            cap = int(pr.count)
            continue
        c.check(st)
        m = int(pr.count)
        if capacity is None:
            c.eps_caps[key] = cap
        return EpsResult(oi[:m], oj[:m], od[:m], m, int(pr.candidates), int(pr.ties))
    raise RuntimeError("join_eps_filtered did not converge on workspace / capacity")


# ---------------------------------------------------------------- measurement
def measure_peaks(device: int | None = None) -> dict:
    """Achievable matrix-core rates (TFLOP/s per operand format, and bf16 at
    the candidate pass's occupancy, with register or LDS operands) and HBM
    copy and read rates (GB/s) of the device, measured by the library's rate
    kernels."""
    c = context(device)
    pk = _lib.dl_peaks()
    c.check(c.L.dl_measure_peaks(c.h, ctypes.byref(pk)))
    return {"fp32": pk.mfma_fp32_tflops, "bf16": pk.mfma_bf16_tflops, "fp16": pk.mfma_fp16_tflops,
            "fp8": pk.mfma_fp8_tflops, "hbm_copy_GBps": pk.hbm_copy_gbps,
            "bf16_16x16x32_2_waves_per_simd": pk.mfma_bf16_2w_tflops,
            "bf16_32x32x16_2_waves_per_simd": pk.mfma_bf16_32x32_2w_tflops, "hbm_read_GBps": pk.hbm_read_gbps,
            "bf16_lds_fed_candidate_loop": pk.mfma_bf16_lds_tflops}


# ---------------------------------------------------------------- top-k
@dataclass
class TopkResult:
    j: torch.Tensor      # int32 (nR, k); -1 (UINT32_MAX) pads
    dist: torch.Tensor   # float32 (nR, k); +inf pads
    band_entries: int
    ties: int


def join_topk(R: torch.Tensor, S: torch.Tensor | None, k: int, exclude_self: bool = False, prec: str = "bf16",
              band_cap: int = 0, stream=None, workspace: Workspace | None = None) -> TopkResult:
    """k nearest rows of S (S=None: of R itself) for every row of R, by
    canonical distance with ties to the smaller index."""
    self_join = S is None
    Sm = R if self_join else S
    c = context(R.device.index)
    ws = workspace or _workspace(R.device)
    p = _lib.PREC[prec]
    nR, nS, d = R.shape[0], Sm.shape[0], R.shape[1]
    oj = torch.empty((nR, k), dtype=torch.int32, device=R.device)
    od = torch.empty((nR, k), dtype=torch.float32, device=R.device)
    info = _lib.dl_topk_info()
    # a call of the same shape starts from the band capacity that sufficed
    # last time instead of growing it again from the default
    key = (nR, nS, d, p, k, self_join, bool(exclude_self))
    asked = band_cap
    if not band_cap:
        band_cap = c.band_caps.get(key, 0)
    for _ in range(6):
        need = c.L.dl_join_topk_workspace(nR, nS, d, p, int(self_join), k, band_cap)
        buf = ws.get(need)
        st = c.L.dl_join_topk(c.h, _mat(R), _mat(Sm), int(self_join), k, int(exclude_self), p, band_cap,
                              ctypes.c_void_p(buf.data_ptr()), buf.numel(), ctypes.c_void_p(oj.data_ptr()),
                              ctypes.c_void_p(od.data_ptr()), ctypes.byref(info), _stream_ptr(stream))
        if c.band_full(st):
            band_cap = max(2 * (band_cap or 1024), 1024)
            continue
        c.check(st)
        if not asked and band_cap:
            c.band_caps[key] = band_cap
        return TopkResult(oj, od, int(info.band_entries), int(info.ties))
    raise RuntimeError("join_topk did not converge on band capacity")



def join_topk_indexed(R: torch.Tensor, S: torch.Tensor | None, k: int, exclude_self: bool = False,
                      prec: str = "bf16", pivots: int = 0, band_cap: int = 0, stream=None,
                      workspace: Workspace | None = None):
    """top-k join with an index built on the fly (each row's k-th distance
    bounded from a sample of S, row-tile balls of that radius, tiles that
    cannot hold a neighbour skipped).  Same result as join_topk; returns
    (TopkResult, IndexInfo)."""
    self_join = S is None
    Sm = R if self_join else S
    c = context(R.device.index)
    ws = workspace or _workspace(R.device)
    p = _lib.PREC[prec]
    nR, nS, d = R.shape[0], Sm.shape[0], R.shape[1]
    oj = torch.empty((nR, k), dtype=torch.int32, device=R.device)
    od = torch.empty((nR, k), dtype=torch.float32, device=R.device)
    info = _lib.dl_topk_info()
    xinfo = _lib.dl_index_info()
    for _ in range(6):
        need = c.L.dl_join_topk_indexed_workspace(nR, nS, d, p, int(self_join), int(exclude_self), k, band_cap,
                                                  pivots)
        buf = ws.get(need)
        st = c.L.dl_join_topk_indexed(c.h, _mat(R), _mat(Sm), int(self_join), k, int(exclude_self), p, band_cap,
                                      pivots, ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                      ctypes.c_void_p(oj.data_ptr()), ctypes.c_void_p(od.data_ptr()),
                                      ctypes.byref(info), ctypes.byref(xinfo), _stream_ptr(stream))
        if c.band_full(st):
            band_cap = max(2 * (band_cap or 1024), 1024)
            continue
        c.check(st)
        return (TopkResult(oj, od, int(info.band_entries), int(info.ties)),
                IndexInfo(int(xinfo.tiles_total), int(xinfo.tiles_computed), int(xinfo.pivots),
                          int(xinfo.ksteps_per_tile), int(xinfo.ksteps_computed)))
    raise RuntimeError("join_topk_indexed did not converge on band capacity")


# ---------------------------------------------------------------- store
class Store:
    """A resident relation: float32 rows (kept alive here) plus their operand
    copy and statistics, built once on the GPU."""

    def __init__(self, base: torch.Tensor, prec: str = "bf16", stream=None):
        self.c = context(base.device.index)
        L = self.c.L
        self.base = base
        self.prec = prec
        self.n, self.d = base.shape
        nbytes = L.dl_store_bytes(self.n, self.d, _lib.PREC[prec])
        self.mem = torch.empty(int(nbytes), dtype=torch.uint8, device=base.device)
        h = ctypes.c_void_p()
        self.c.check(L.dl_store_create(self.c.h, _mat(base), _lib.PREC[prec], ctypes.c_void_p(self.mem.data_ptr()),
                                       nbytes, ctypes.byref(h), _stream_ptr(stream)))
        self.h = h

    @classmethod
    def featurize(cls, pixels: torch.Tensor, bins: int = 8, prec: str = "bf16", boxes: torch.Tensor | None = None,
                  stream=None) -> "Store":
        """Featurise and materialise in one pass: the colour histograms of
        uint8 (n, h, w, 3) patches, or of boxes (int32 (m, 5)) over uint8
        (nframes, h, w, 3) frames, become the store's float32 rows (kept in
        self.base) and its operand copy, without reading the rows back."""
        if pixels.dtype != torch.uint8 or pixels.dim() != 4 or pixels.shape[3] != 3 or not pixels.is_cuda:
            raise TypeError("pixels must be a (n, h, w, 3) uint8 CUDA tensor")
        self = cls.__new__(cls)
        self.c = context(pixels.device.index)
        L = self.c.L
        pixels = pixels.contiguous()
        n, h, w, _ = pixels.shape
        bptr, nb = None, 0
        if boxes is not None:
            boxes = boxes.to(device=pixels.device, dtype=torch.int32).contiguous().reshape(-1, 5)
            bptr, nb = ctypes.c_void_p(boxes.data_ptr()), boxes.shape[0]
        rows = nb if boxes is not None else n
        self.base = torch.empty((rows, bins ** 3), dtype=torch.float32, device=pixels.device)
        self.prec = prec
        self.n, self.d = self.base.shape
        nbytes = L.dl_store_bytes(self.n, self.d, _lib.PREC[prec])
        self.mem = torch.empty(int(nbytes), dtype=torch.uint8, device=pixels.device)
        hd = ctypes.c_void_p()
        self.c.check(L.dl_store_featurize_rgb8(self.c.h, ctypes.c_void_p(pixels.data_ptr()), n, h, w, bptr, nb, bins,
                                               _lib.PREC[prec], ctypes.c_void_p(self.base.data_ptr()),
                                               ctypes.c_void_p(self.mem.data_ptr()), nbytes, ctypes.byref(hd),
                                               _stream_ptr(stream)))
        self.h = hd
        return self

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.c.L.dl_store_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def join_eps_self(self, eps: float, max_candidates: int | None = None, stream=None,
                      workspace: Workspace | None = None, out: tuple | None = None) -> EpsResult:
        """eps self-join (i < j) of the store's rows on its operand copy."""
        c, L = self.c, self.c.L
        ws = workspace or _workspace(self.base.device)
        if max_candidates is None:
            max_candidates = max(1 << 20, 4 * self.n)
        # a call with the same eps starts from the output size that sufficed
        caps = self.__dict__.setdefault("_eps_caps", {})
        cap = out[0].numel() if out is not None else max(1 << 16, 2 * self.n, caps.get(float(eps), 0))
        for _ in range(8):
            buf = ws.get(L.dl_join_eps_store_self_workspace(self.h, max_candidates))
            if out is not None and out[0].numel() >= cap:
                oi, oj, od = out
            else:
                oi = torch.empty(cap, dtype=torch.int32, device=self.base.device)
                oj = torch.empty(cap, dtype=torch.int32, device=self.base.device)
                od = torch.empty(cap, dtype=torch.float32, device=self.base.device)
            pr = _lib.dl_pairs(oi.data_ptr(), oj.data_ptr(), od.data_ptr(), cap, 0, 0, 0)
            st = L.dl_join_eps_store_self(c.h, self.h, float(eps), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                          ctypes.byref(pr), _stream_ptr(stream))
            if st == _lib.DL_ERR_WORKSPACE:
                max_candidates = max(2 * max_candidates, int(pr.candidates * 1.25) + 1024)
                continue
            if st == _lib.DL_ERR_CAPACITY:
                cap = int(pr.count)
                out = None
                continue
            c.check(st)
            m = int(pr.count)
            caps[float(eps)] = cap
            return EpsResult(oi[:m], oj[:m], od[:m], m, int(pr.candidates), int(pr.ties))
        raise RuntimeError("join_eps_self (store) did not converge")

    def join_eps(self, R: torch.Tensor, eps: float, max_candidates: int | None = None, stream=None,
                 workspace: Workspace | None = None) -> EpsResult:
        c, L = self.c, self.c.L
        ws = workspace or _workspace(R.device)
        nR = R.shape[0]
        if max_candidates is None:
            max_candidates = max(1 << 20, 64 * nR)
        cap = max(1 << 16, 16 * nR)
        for _ in range(10):
            buf = ws.get(L.dl_join_eps_store_workspace(nR, self.h, max_candidates))
            oi = torch.empty(cap, dtype=torch.int32, device=R.device)
            oj = torch.empty(cap, dtype=torch.int32, device=R.device)
            od = torch.empty(cap, dtype=torch.float32, device=R.device)
            pr = _lib.dl_pairs(oi.data_ptr(), oj.data_ptr(), od.data_ptr(), cap, 0, 0, 0)
            st = L.dl_join_eps_store(c.h, _mat(R), self.h, float(eps), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                     ctypes.byref(pr), _stream_ptr(stream))
            if st == _lib.DL_ERR_WORKSPACE:
                max_candidates = max(2 * max_candidates, int(pr.candidates * 1.25) + 1024)
                continue
            if st == _lib.DL_ERR_CAPACITY:
                cap = int(pr.count)
                continue
            c.check(st)
            m = int(pr.count)
            return EpsResult(oi[:m], oj[:m], od[:m], m, int(pr.candidates), int(pr.ties))
        raise RuntimeError("join_eps (store) did not converge")

    def join_topk(self, R: torch.Tensor, k: int, band_cap: int = 0, stream=None,
                  workspace: Workspace | None = None) -> TopkResult:
        c, L = self.c, self.c.L
        ws = workspace or _workspace(R.device)
        nR = R.shape[0]
        oj = torch.empty((nR, k), dtype=torch.int32, device=R.device)
        od = torch.empty((nR, k), dtype=torch.float32, device=R.device)
        info = _lib.dl_topk_info()
        for _ in range(6):
            buf = ws.get(L.dl_join_topk_store_workspace(nR, self.h, k, band_cap))
            st = L.dl_join_topk_store(c.h, _mat(R), self.h, k, band_cap, ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                      ctypes.c_void_p(oj.data_ptr()), ctypes.c_void_p(od.data_ptr()), ctypes.byref(info),
                                      _stream_ptr(stream))
            if c.band_full(st):
                band_cap = max(2 * (band_cap or 1024), 1024)
                continue
            c.check(st)
            return TopkResult(oj, od, int(info.band_entries), int(info.ties))
        raise RuntimeError("join_topk (store) did not converge")


class _DeviceView:
    """Zero-copy view of library-owned device memory for torch.as_tensor."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr or 0), False),
                                         "version": 2, "strides": None}


def _view(ptr, shape, typestr, device):
    if int(ptr or 0) == 0 or 0 in shape:
        dt = {"<u4": torch.int32, "<f4": torch.float32}[typestr]
        return torch.empty(shape, dtype=dt, device=device)
    return torch.as_tensor(_DeviceView(ptr, shape, typestr), device=device)


class Server:
    """Batching request loop over a Store (see dl_server_* in dlmi.h)."""

    def __init__(self, store: Store, arena_bytes: int, n_streams: int = 2, max_batch_requests: int = 64,
                 max_batch_rows: int = 1 << 16, pairs_per_row: int = 64, band_cap: int = 0, small_rows: int = 0):
        self.store = store
        self.c = store.c
        self.L = self.c.L
        self.device = store.base.device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        cfg = _lib.dl_server_config(n_streams, max_batch_requests, max_batch_rows, pairs_per_row, band_cap, small_rows)
        h = ctypes.c_void_p()
        st = self.L.dl_server_create(self.device.index or 0, store.h, ctypes.byref(cfg),
                                     ctypes.c_void_p(self.arena.data_ptr()), self.arena.numel(), ctypes.byref(h))
        if st != _lib.DL_OK:
            raise _lib.DLError(st, "dl_server_create failed")
        self.h = h
        self._live = {}

    def submit(self, query: torch.Tensor, mode: str, eps: float = 0.0, k: int = 10, sync: bool = True) -> int:
        """Queue a request; `query` must be complete on the device (with
        sync=True this call waits for the current stream) and is kept alive
        until completion."""
        if sync:
            torch.cuda.current_stream().synchronize()
        m = _lib.DL_MODE_EPS if mode == "eps" else _lib.DL_MODE_TOPK
        rq = _lib.dl_request(_mat(query), m, float(eps), int(k))
        t = ctypes.c_uint64()
        st = self.L.dl_server_submit(self.h, ctypes.byref(rq), ctypes.byref(t))
        if st != _lib.DL_OK:
            raise _lib.DLError(st, "submit rejected")
        self._live[t.value] = query
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1, fetch: bool = True) -> dict:
        """Wait for a request, copy its result into torch tensors (unless
        fetch=False), and release it."""
        r = _lib.dl_result()
        st = self.L.dl_server_wait(self.h, ticket, timeout_ms, ctypes.byref(r))
        if st != _lib.DL_OK:
            raise _lib.DLError(st, "wait failed")
        out = {"status": r.status, "mode": "eps" if r.mode == _lib.DL_MODE_EPS else "topk", "rows": r.rows,
               "latency_ms": r.latency_ms, "queued_ms": r.queued_ms, "batch_id": r.batch_id,
               "batch_requests": r.batch_requests}
        if r.status == _lib.DL_OK and r.mode == _lib.DL_MODE_EPS:
            out["count"] = int(r.count)
        if r.status == _lib.DL_OK and fetch:
            if r.mode == _lib.DL_MODE_EPS:
                n = int(r.count)
                out["i"] = _view(r.i, (n,), "<u4", self.device).clone()
                out["j"] = _view(r.j, (n,), "<u4", self.device).clone()
                out["dist"] = _view(r.dist, (n,), "<f4", self.device).clone()
                out["count"] = n
            else:
                out["j"] = _view(r.j, (int(r.rows), int(r.k)), "<u4", self.device).clone()
                out["dist"] = _view(r.dist, (int(r.rows), int(r.k)), "<f4", self.device).clone()
            torch.cuda.current_stream().synchronize()  # copies done before the memory is reused
        self.L.dl_server_release(self.h, ticket)
        self._live.pop(ticket, None)
        return out

    def cancel(self, ticket: int) -> bool:
        return self.L.dl_server_cancel(self.h, ticket) == _lib.DL_OK

    def stats(self) -> dict:
        s = _lib.dl_server_info()
        self.L.dl_server_stats(self.h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def reset_stats(self):
        self.L.dl_server_reset_stats(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.L.dl_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
