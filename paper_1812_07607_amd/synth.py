"""Seeded synthetic inputs for the patch-matching workloads.

This module only draws random inputs (patches, feature vectors, sampled pair
indices, request streams).  It holds none of the featurisation or join
arithmetic, so both the GPU path and the CPU oracle can take their inputs
from it.  The paper's own datasets (a personal photo collection, traffic-camera
video and football clips; section "Datasets") are not available; the
generators below stand in for their shape: clustered colour histograms of
small crops for near-duplicate matching (queries q1 and q4), and clustered
unit-norm embeddings for the larger joins.

Every generator is a pure function of its seed.  Large arrays are produced in
fixed-size chunks, each from its own child of the root SeedSequence, so the
output does not depend on the number of worker threads.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1 << 16  # rows per independently seeded chunk


def _rng(seed, *path):
    ss = np.random.SeedSequence(seed)
    for p in path:
        ss = ss.spawn(p + 1)[p]
    return np.random.default_rng(ss)


def _workers():
    import os
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n, fill, seed, tag):
    """Run fill(lo, hi, rng) over [0, n) in CHUNK-row pieces, in parallel."""
    nchunks = (n + CHUNK - 1) // CHUNK
    root = np.random.SeedSequence([seed, tag])
    kids = root.spawn(nchunks) if nchunks else []

    def run(c):
        lo, hi = c * CHUNK, min(n, (c + 1) * CHUNK)
        fill(lo, hi, np.random.default_rng(kids[c]))

    if nchunks <= 1:
        for c in range(nchunks):
            run(c)
    else:
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(run, range(nchunks)))


# ---------------------------------------------------------------------------
# Patches: uint8 RGB crops, HWC, R,G,B per pixel.
# ---------------------------------------------------------------------------
def patches_palette(n, h=32, w=32, n_colours=16, sigma=20.0, seed=202):
    """n patches of h x w RGB pixels.  Each patch picks one of n_colours base
    colours (uniform over {0..255}^3, drawn once from the seed); each pixel and
    channel is round(base + N(0, sigma^2)) clipped to [0, 255].

    Returns (patches uint8 (n,h,w,3), colour index int32 (n,)).
    """
    rng = _rng(seed, 0)
    base = rng.integers(0, 256, size=(n_colours, 3)).astype(np.float32)
    colour = rng.integers(0, n_colours, size=n).astype(np.int32)
    out = np.empty((n, h, w, 3), np.uint8)

    def fill(lo, hi, r):
        z = r.standard_normal((hi - lo, h, w, 3), dtype=np.float32)
        z *= np.float32(sigma)
        z += base[colour[lo:hi]][:, None, None, :]
        np.rint(z, out=z)
        np.clip(z, 0, 255, out=z)
        out[lo:hi] = z.astype(np.uint8)

    _chunked(n, fill, seed, 1)
    return out, colour


def frames_with_boxes(nframes, height, width, nboxes, n_colours=16, sigma=20.0, min_side=4, max_side=96,
                      seed=606):
    """Frames with coloured objects, and bounding boxes over them.

    Each frame is uniform noise with up to 12 axis-aligned rectangles, each
    filled with one of n_colours base colours (drawn once from the seed) plus
    N(0, sigma^2) noise per pixel and channel (rounded, clipped to 0..255).
    Each box covers one object, cut at the frame's border, or, one time in
    four, a random region; sides are log-uniform in [min_side, max_side], so
    pixel counts are ragged and mostly not powers of two.

    Returns (frames uint8 (nframes, height, width, 3), boxes int32 (nboxes, 5)
    as (frame, x0, y0, x1, y1) with x0 <= x < x1, y0 <= y < y1).
    """
    rng = _rng(seed, 70)
    base = rng.integers(0, 256, size=(n_colours, 3)).astype(np.float32)
    frames = rng.integers(0, 256, size=(nframes, height, width, 3), dtype=np.uint8)
    hi = min(max_side, height, width)
    lo = min(min_side, hi)

    def side():
        return int(np.clip(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi)))), lo, hi))

    objects = []
    for f in range(nframes):
        for _ in range(int(rng.integers(1, 13))):
            w, h = side(), side()
            x0, y0 = int(rng.integers(0, width - w + 1)), int(rng.integers(0, height - h + 1))
            z = base[int(rng.integers(0, n_colours))] + sigma * rng.standard_normal((h, w, 3), dtype=np.float32)
            frames[f, y0:y0 + h, x0:x0 + w] = np.clip(np.rint(z), 0, 255).astype(np.uint8)
            objects.append((f, x0, y0, x0 + w, y0 + h))
    boxes = np.empty((nboxes, 5), np.int32)
    for b in range(nboxes):
        if objects and rng.random() < 0.75:
            boxes[b] = objects[int(rng.integers(0, len(objects)))]
        else:
            w, h = side(), side()
            f = int(rng.integers(0, nframes))
            x0, y0 = int(rng.integers(0, width - w + 1)), int(rng.integers(0, height - h + 1))
            boxes[b] = (f, x0, y0, x0 + w, y0 + h)
    return frames, boxes


def patches_uniform(n, h, w, seed):
    """n patches of independent uniform uint8 pixels."""
    return _rng(seed, 2).integers(0, 256, size=(n, h, w, 3), dtype=np.uint8)


# ---------------------------------------------------------------------------
# Feature vectors.
# ---------------------------------------------------------------------------
def dirichlet_clusters(n, d=64, n_centres=20, alpha=0.5, mix=0.25, seed=101, stream=0):
    """L1-normalised vectors around n_centres Dirichlet(alpha) centres.

    Centres c_m ~ Dir(alpha 1_d) are drawn from the seed alone (shared by all
    streams); row x = (1-mix) c_m + mix u with m uniform and u ~ Dir(alpha 1_d),
    renormalised to unit L1 mass in float64 and rounded to float32.  Different
    `stream` values give independent rows around the same centres (R and S).
    """
    rc = _rng(seed, 0)
    centres = rc.dirichlet(np.full(d, alpha), size=n_centres)
    r = _rng(seed, 1 + stream)
    m = r.integers(0, n_centres, size=n)
    u = r.dirichlet(np.full(d, alpha), size=n)
    x = (1.0 - mix) * centres[m] + mix * u
    x /= x.sum(axis=1, keepdims=True)
    return x.astype(np.float32)


def gaussian_mixture_unit(n, d, n_centres, sigma=0.05, seed=303, stream=0):
    """Unit-norm float32 rows of a Gaussian mixture on the sphere.

    Centres mu_m = g / |g| with g ~ N(0, I_d), drawn from the seed alone;
    row x = (mu_m + sigma z) / |mu_m + sigma z| with m uniform, z ~ N(0, I_d).
    Normalisation is done in float64 per chunk, then rounded to float32.
    """
    rc = _rng(seed, 0)
    centres = rc.standard_normal((n_centres, d))
    centres /= np.linalg.norm(centres, axis=1, keepdims=True)
    out = np.empty((n, d), np.float32)

    def fill(lo, hi, r):
        m = r.integers(0, n_centres, size=hi - lo)
        x = centres[m] + sigma * r.standard_normal((hi - lo, d))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[lo:hi] = x

    _chunked(n, fill, seed, 10 + stream)
    return out


def block_sparse_rows(n, d=512, groups=8, sigma=0.1, faint=0.1, faint_norm=0.05, seed=0, stream=0):
    """Rows nonzero only inside one of `groups` equal blocks of coordinates
    (like colour histograms whose mass sits in a few bins): row x of group g
    is (mu_g + sigma z) restricted to block g, normalised to unit length, mu_g
    a unit vector inside block g drawn from the seed alone; a fraction
    `faint` of the rows is then scaled to length `faint_norm`, so rows of
    different blocks can still lie close together.  float32."""
    rc = _rng(seed, 0)
    w = d // groups
    mu = rc.standard_normal((groups, w))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    r = _rng(seed, 40 + stream)
    g = r.integers(0, groups, size=n)
    x = mu[g] + sigma * r.standard_normal((n, w))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    x[r.random(n) < faint] *= faint_norm
    out = np.zeros((n, d), np.float32)
    for k in range(groups):
        rows = np.nonzero(g == k)[0]
        out[rows, k * w:(k + 1) * w] = x[rows]
    return out


def uniform_rows(n, d, lo=-1.0, hi=1.0, seed=0, stream=0):
    """Independent uniform float32 rows (no structure)."""
    return _rng(seed, 20 + stream).uniform(lo, hi, size=(n, d)).astype(np.float32)


def integer_grid_rows(n, d, levels=3, scale=0.25, seed=0, stream=0):
    """Rows on a coarse integer grid times `scale`; many exactly equal
    distances, so ties at the eps boundary and at the k-th neighbour are
    frequent."""
    r = _rng(seed, 30 + stream)
    return (r.integers(0, levels, size=(n, d)) * scale).astype(np.float32)


# ---------------------------------------------------------------------------
# Random draws of the workload definition (passed to both sides as inputs).
# ---------------------------------------------------------------------------
def sample_pairs(n_r, n_s, m, self_join, seed):
    """m pairs drawn uniformly with replacement.  For a self-join the pair is
    drawn with i != j and returned ordered as (min, max)."""
    r = _rng(seed, 40)
    i = r.integers(0, n_r, size=m, dtype=np.int64)
    if self_join:
        j = r.integers(0, n_s - 1, size=m, dtype=np.int64)
        j = j + (j >= i)  # uniform over {0..n-1} \ {i}
        lo, hi = np.minimum(i, j), np.maximum(i, j)
        return lo, hi
    j = r.integers(0, n_s, size=m, dtype=np.int64)
    return i, j


def order_statistic(values, q):
    """Lower order statistic: sorted(values)[ceil(q * M) - 1]."""
    v = np.sort(np.asarray(values))
    idx = max(0, int(math.ceil(q * len(v))) - 1)
    return v[idx]


def sample_rows(n, m, seed):
    """m distinct row indices in [0, n), increasing."""
    r = _rng(seed, 50)
    return np.sort(r.choice(n, size=min(m, n), replace=False)).astype(np.int64)


def request_stream(n_requests, rate_hz, max_rows=50000, seed=505):
    """Serving workload: Poisson arrivals at rate_hz; sizes
    round(exp(U(0, ln max_rows))) (log-uniform in 1..max_rows); mode
    eps / top-10 with probability 1/2 each.  Returns (arrival_s float64,
    rows int64, is_topk bool)."""
    r = _rng(seed, 60)
    gaps = r.exponential(1.0 / rate_hz, size=n_requests)
    arrival = np.cumsum(gaps) - gaps[0]
    rows = np.rint(np.exp(r.uniform(0.0, math.log(max_rows), size=n_requests))).astype(np.int64)
    rows = np.clip(rows, 1, max_rows)
    is_topk = r.random(n_requests) < 0.5
    return arrival, rows, is_topk


# ---------------------------------------------------------------------------
# The five workload configurations (sizes as named; `scale` shrinks them for
# tests).
# ---------------------------------------------------------------------------
CONFIG_SEEDS = {1: 101, 2: 202, 3: 303, 4: 404, 5: 505}


def config1(scale=1.0):
    """eps-join of 2,000 x 2,000 L1-normalised vectors, d = 64, 20 Dirichlet
    centres; eps is the 0.1% order statistic of 10,000 sampled pair
    distances."""
    n = max(2, int(2000 * scale))
    s = CONFIG_SEEDS[1]
    R = dirichlet_clusters(n, 64, 20, 0.5, seed=s, stream=0)
    S = dirichlet_clusters(n, 64, 20, 0.5, seed=s, stream=1)
    pi, pj = sample_pairs(n, n, 10000, False, s)
    return {"R": R, "S": S, "pairs": (pi, pj), "q": 0.001}


def config2(scale=1.0):
    """Featurise 100,000 RGB 32x32 patches (16 base colours + N(0, 20^2)
    noise) into 8x8x8 histograms, then eps self-join at the 0.01% order
    statistic of 1,000,000 sampled i<j pair distances."""
    n = max(2, int(100000 * scale))
    s = CONFIG_SEEDS[2]
    patches, colour = patches_palette(n, 32, 32, 16, 20.0, seed=s)
    pi, pj = sample_pairs(n, n, 1000000 if scale >= 1.0 else max(1000, int(1000000 * scale)), True, s)
    return {"patches": patches, "colour": colour, "pairs": (pi, pj), "q": 0.0001}


def config3(scale=1.0):
    """1,000,000 x 1,000,000 unit-norm vectors, d = 128, 1,000 centres,
    sigma = 0.05; top-10 and eps-join."""
    n = max(16, int(1000000 * scale))
    s = CONFIG_SEEDS[3]
    R = gaussian_mixture_unit(n, 128, 1000, 0.05, seed=s, stream=0)
    S = gaussian_mixture_unit(n, 128, 1000, 0.05, seed=s, stream=1)
    return {"R": R, "S": S, "k": 10}


def config4(scale=1.0):
    """Store of 4,000,000 unit-norm vectors, d = 256, 4,096 centres; 50,000
    queries from the same mixture; top-32 with FP8 candidates."""
    ns = max(64, int(4000000 * scale))
    nq = max(16, int(50000 * scale))
    s = CONFIG_SEEDS[4]
    S = gaussian_mixture_unit(ns, 256, 4096, 0.05, seed=s, stream=0)
    Q = gaussian_mixture_unit(nq, 256, 4096, 0.05, seed=s, stream=1)
    return {"S": S, "Q": Q, "k": 32}


def config5(scale=1.0):
    """Serving: store of 8,000,000 unit-norm vectors, d = 128, 1,000 centres;
    requests log-uniform in 1..50,000 rows, half eps-join and half top-10."""
    ns = max(64, int(8000000 * scale))
    s = CONFIG_SEEDS[5]
    S = gaussian_mixture_unit(ns, 128, 1000, 0.05, seed=s, stream=0)
    return {"S": S, "k": 10, "seed": s}


def queries_for_store(n, d, n_centres, seed, stream=1):
    return gaussian_mixture_unit(n, d, n_centres, 0.05, seed=seed, stream=stream)
