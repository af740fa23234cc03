"""The seeded input generators are deterministic and have the stated shapes."""
import hashlib

import numpy as np

from paper_1812_07607_amd import synth


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_deterministic_and_thread_independent(monkeypatch):
    a = synth.gaussian_mixture_unit(3 * synth.CHUNK + 5, 8, 7, seed=1)
    monkeypatch.setattr(synth, "_workers", lambda: 1)
    b = synth.gaussian_mixture_unit(3 * synth.CHUNK + 5, 8, 7, seed=1)
    assert digest(a) == digest(b)
    assert digest(a) != digest(synth.gaussian_mixture_unit(3 * synth.CHUNK + 5, 8, 7, seed=2))


def test_patches_palette():
    p, c = synth.patches_palette(300, 32, 32, 16, 20.0, seed=202)
    p2, c2 = synth.patches_palette(300, 32, 32, 16, 20.0, seed=202)
    assert p.shape == (300, 32, 32, 3) and p.dtype == np.uint8
    assert digest(p, c) == digest(p2, c2)
    assert set(np.unique(c)) <= set(range(16))
    # per-patch channel means sit near one of the 16 base colours
    means = p.reshape(300, -1, 3).mean(axis=1)
    assert len(np.unique(np.round(means[c == c[0]] / 16))) <= 8


def test_vector_generators():
    x = synth.dirichlet_clusters(500, 64, 20, seed=101)
    assert x.dtype == np.float32 and x.shape == (500, 64)
    assert np.allclose(x.sum(axis=1), 1.0, atol=1e-5) and np.all(x >= 0)
    u = synth.gaussian_mixture_unit(1000, 128, 10, seed=3)
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-5)


def test_sample_pairs_self():
    i, j = synth.sample_pairs(50, 50, 10000, True, seed=1)
    assert np.all(i < j) and i.min() >= 0 and j.max() < 50


def test_order_statistic():
    v = np.arange(10000)[::-1].astype(float)
    assert synth.order_statistic(v, 0.001) == 9.0
    assert synth.order_statistic(v, 0.0001) == 0.0


def test_request_stream():
    t, rows, topk = synth.request_stream(2000, 100.0, seed=5)
    assert np.all(np.diff(t) >= 0) and rows.min() >= 1 and rows.max() <= 50000
    assert 0.4 < topk.mean() < 0.6
