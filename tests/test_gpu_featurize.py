"""GPU parity of the colour-histogram kernels against the oracle: bit-exact
(patches, crops of frames, and the fused featurise-into-store pass)."""
import numpy as np
import pytest
import torch

from gpu_util import assert_eps_equal, assert_topk_equal, dev, host
from paper_1812_07607_amd import ops, synth
from paper_1812_07607_amd._lib import DL_ERR_INVALID, DLError

pytestmark = pytest.mark.gpu


def test_full_size_palette_patches(orc):
    """100,000 patches of 32x32 (the featurise-and-self-join workload)."""
    cfg = synth.config2(1.0)
    patches = cfg["patches"]
    got = host(ops.featurize_rgb8(dev(patches), 8))
    ref = orc.hist_rgb8(patches, 8)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("hw", [(1, 1), (7, 5), (32, 32), (17, 31), (64, 48), (4, 4)])
@pytest.mark.parametrize("bins", [8, 4, 16])
def test_shapes_and_bins(orc, hw, bins):
    for n in (0, 1, 3, 1001):
        p = synth.patches_uniform(n, hw[0], hw[1], seed=n + 7)
        got = host(ops.featurize_rgb8(dev(p), bins))
        assert np.array_equal(got, orc.hist_rgb8(p, bins)), (n, hw, bins)


def test_unaligned_patch_buffer(orc):
    p = synth.patches_uniform(41, 32, 32, seed=3)
    flat = torch.zeros(41 * 32 * 32 * 3 + 1, dtype=torch.uint8, device="cuda")
    flat[1:] = dev(p.reshape(-1))
    view = flat[1:].view(41, 32, 32, 3)  # start is 1 byte past a 16-byte boundary
    got = host(ops.featurize_rgb8(view, 8))
    assert np.array_equal(got, orc.hist_rgb8(p, 8))


def test_extreme_colours(orc):
    # every pixel on a bin edge or at 0 / 255
    vals = np.array([0, 31, 32, 63, 64, 223, 224, 255], np.uint8)
    rng = np.random.default_rng(0)
    p = vals[rng.integers(0, len(vals), size=(64, 16, 16, 3))]
    got = host(ops.featurize_rgb8(dev(p), 8))
    assert np.array_equal(got, orc.hist_rgb8(p, 8))


def test_rejects_bad_arguments():
    with pytest.raises(Exception):
        ops.featurize_rgb8(dev(np.zeros((2, 4, 4, 3), np.uint8)), 3)
    with pytest.raises(TypeError):
        ops.featurize_rgb8(dev(np.zeros((2, 4, 4), np.uint8)), 8)


# ----------------------------------------------------------------- crops
def test_crops_bit_exact(orc):
    """Boxes over 360x640 frames with ragged, mostly non-power-of-two pixel
    counts (and a whole frame, a single pixel, a one-pixel-wide strip)."""
    frames, boxes = synth.frames_with_boxes(6, 360, 640, 3000, seed=606)
    boxes[0] = (2, 0, 0, 640, 360)
    boxes[1] = (5, 639, 359, 640, 360)
    boxes[2] = (1, 17, 0, 18, 360)
    ref = orc.hist_crops(frames, boxes, 8)
    got = host(ops.featurize_crops_rgb8(dev(frames), dev(boxes), 8))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("bins", [4, 16])
def test_crops_other_bins_and_odd_frames(orc, bins):
    frames, boxes = synth.frames_with_boxes(3, 37, 53, 400, min_side=1, max_side=37, seed=bins)
    ref = orc.hist_crops(frames, boxes, bins)
    got = host(ops.featurize_crops_rgb8(dev(frames), dev(boxes), bins))
    assert np.array_equal(got, ref)


def test_crops_outside_the_frame_are_rejected(orc):
    frames, boxes = synth.frames_with_boxes(2, 40, 50, 8, seed=3)
    bad = boxes.copy()
    bad[3] = (1, 45, 10, 51, 20)  # past the right edge
    with pytest.raises(DLError) as e:
        ops.featurize_crops_rgb8(dev(frames), dev(bad), 8)
    assert e.value.status == DL_ERR_INVALID
    # the valid boxes still get their histograms, the bad one zeros
    out = torch.full((8, 512), 7.0, device="cuda")
    with pytest.raises(DLError):
        ops.featurize_crops_rgb8(dev(frames), dev(bad), 8, out=out)
    ref = orc.hist_crops(frames, np.delete(bad, 3, axis=0), 8)
    got = host(out)
    assert np.array_equal(np.delete(got, 3, axis=0), ref) and not got[3].any()


# ------------------------------------------- featurise into a store (fused)
@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp8", "fp32"])
def test_store_featurize_patches_and_self_join(orc, prec):
    """Histograms written by the fused featurise-and-prep pass equal the
    oracle's; the store's self-join (on its operand copy, no prep) equals the
    oracle's eps self-join and the plain join."""
    cfg = synth.config2(0.05)
    Href = orc.hist_rgb8(cfg["patches"], 8)
    st = ops.Store.featurize(dev(cfg["patches"]), 8, prec)
    assert np.array_equal(host(st.base), Href)
    pi, pj = cfg["pairs"]
    eps = float(np.sqrt(synth.order_statistic(orc.pair_d2(Href, Href, pi, pj), cfg["q"])))
    ref = orc.eps_join(Href, None, eps)
    got = st.join_eps_self(eps)
    assert_eps_equal(got, ref, 512, "store self-join/" + prec)
    plain = ops.join_eps(st.base, None, eps, prec)
    assert torch.equal(got.i, plain.i) and torch.equal(got.j, plain.j) and torch.equal(got.dist, plain.dist)
    # and the store serves probes like one built from the rows
    Q = Href[:300]
    rj, _, rd = orc.topk(Q, Href, 5)
    assert_topk_equal(st.join_topk(dev(Q), 5), rj, rd, 512, "fused store top-5/" + prec)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_store_featurize_crops(orc, prec):
    frames, boxes = synth.frames_with_boxes(5, 200, 300, 1500, seed=7)
    Href = orc.hist_crops(frames, boxes, 8)
    st = ops.Store.featurize(dev(frames), 8, prec, boxes=dev(boxes))
    assert np.array_equal(host(st.base), Href)
    pairs = synth.sample_pairs(1500, 1500, 20000, True, seed=8)
    eps = float(np.sqrt(synth.order_statistic(orc.pair_d2(Href, Href, *pairs), 0.01)))
    assert_eps_equal(st.join_eps_self(eps), orc.eps_join(Href, None, eps), 512, "crop store self-join/" + prec)
