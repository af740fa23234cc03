"""Pins for the oracle's colour histogram (section "Visual ETL", Transformers).

The oracle is checked against things other than itself: a hand-computed
example, numpy's histogramdd (an independent binning routine), and
invariants (mass, permutation, bin edges)."""
import numpy as np
import pytest

from conftest import read_golden


def histogramdd_reference(patches, bins):
    """Counts via numpy.histogramdd with uniform edges 0, 256/bins, ..., 256."""
    n = patches.shape[0]
    edges = np.linspace(0, 256, bins + 1)
    out = np.empty((n, bins ** 3), np.int64)
    for p in range(n):
        px = patches[p].reshape(-1, 3).astype(np.float64)
        c, _ = np.histogramdd(px, bins=(edges, edges, edges))
        out[p] = c.astype(np.int64).reshape(-1)  # C order: r major, then g, then b
    return out


def test_hand_example(orc):
    rows = read_golden("hist_2x2.txt")
    bins = int([r for r in rows if r[0] == "bins"][0][1])
    h, w = map(int, [r for r in rows if r[0] == "size"][0][1:])
    px = np.array([list(map(int, r[1:])) for r in rows if r[0] == "pixel"], np.uint8)
    patch = px.reshape(1, h, w, 3)
    expect = np.zeros(bins ** 3, np.float32)
    for r in rows:
        if r[0] == "expect":
            expect[int(r[1])] = float(r[2])
    got = orc.hist_rgb8(patch, bins)
    assert got.shape == (1, bins ** 3)
    assert np.array_equal(got[0], expect)


@pytest.mark.parametrize("bins", [8, 4, 16, 2])
@pytest.mark.parametrize("hw", [(32, 32), (7, 5), (1, 1), (17, 31)])
def test_matches_histogramdd(orc, bins, hw):
    rng = np.random.default_rng(bins * 100 + hw[0])
    patches = rng.integers(0, 256, size=(6, hw[0], hw[1], 3), dtype=np.uint8)
    h, cnt = orc.hist_rgb8(patches, bins, counts=True)
    ref = histogramdd_reference(patches, bins)
    assert np.array_equal(cnt, ref)
    npx = hw[0] * hw[1]
    # L1 normalisation: one correctly rounded division per bin
    assert np.array_equal(h, (ref.astype(np.float64) / npx).astype(np.float32))


def test_single_colour_patch(orc):
    rng = np.random.default_rng(7)
    for _ in range(20):
        c = rng.integers(0, 256, size=3)
        patch = np.broadcast_to(c.astype(np.uint8), (1, 8, 8, 3)).copy()
        h = orc.hist_rgb8(patch, 8)[0]
        ref = histogramdd_reference(patch, 8)[0]
        assert h.max() == 1.0 and np.count_nonzero(h) == 1
        assert np.argmax(h) == np.argmax(ref)


def test_bin_edges(orc):
    # values on either side of the first, an interior and the last edge
    vals = [0, 31, 32, 223, 224, 255]
    for ch in range(3):
        for v in vals:
            px = np.zeros((1, 1, 1, 3), np.uint8)
            px[0, 0, 0, ch] = v
            h = orc.hist_rgb8(px, 8)[0]
            ref = histogramdd_reference(px, 8)[0]
            assert np.argmax(h) == np.argmax(ref), (ch, v)
    # 31 and 32 fall in different bins, 223 and 224 too; 0 and 31 share one
    def binof(v):
        return int(np.argmax(orc.hist_rgb8(np.full((1, 1, 1, 3), v, np.uint8), 8)[0]))
    assert binof(0) == binof(31) != binof(32)
    assert binof(223) != binof(224) == binof(255)


def test_mass_and_permutation(orc):
    rng = np.random.default_rng(11)
    patches = rng.integers(0, 256, size=(5, 32, 32, 3), dtype=np.uint8)
    h, cnt = orc.hist_rgb8(patches, 8, counts=True)
    assert np.all(cnt.sum(axis=1) == 32 * 32)
    # 1024 pixels: every bin is a multiple of 2^-10, so the float32 sum is exact
    assert np.all(h.astype(np.float32).sum(axis=1, dtype=np.float32) == np.float32(1.0))
    for p in range(5):
        flat = patches[p].reshape(-1, 3)
        perm = flat[rng.permutation(flat.shape[0])].reshape(1, 32, 32, 3)
        assert np.array_equal(orc.hist_rgb8(perm, 8)[0], h[p])


def test_nonpow2_pixel_count_rounding(orc):
    # 3 pixels in one bin out of 7: value is the float32 nearest to 3/7
    px = np.zeros((1, 1, 7, 3), np.uint8)
    px[0, 0, 3:, 0] = 200
    h = orc.hist_rgb8(px, 8)[0]
    assert h[0] == np.float32(3 / 7) and h[6 * 64] == np.float32(4 / 7)


def test_empty_batch(orc):
    h = orc.hist_rgb8(np.zeros((0, 4, 4, 3), np.uint8), 8)
    assert h.shape == (0, 512)


def test_rejects_bad_bins(orc):
    with pytest.raises(ValueError):
        orc.hist_rgb8(np.zeros((1, 2, 2, 3), np.uint8), 3)


# ----------------------------------------------------------------- crops
def read_crop_golden():
    rows = read_golden("crop_hand.txt")
    bins = int([r for r in rows if r[0] == "bins"][0][1])
    h, w = map(int, [r for r in rows if r[0] == "frame"][0][1:])
    px = [list(map(int, r[1:])) for r in rows if r[0] == "row"]
    frame = np.array(px, np.uint8).reshape(1, h, w, 3)
    boxes, expects = [], []
    for r in rows:
        if r[0] == "box":
            boxes.append(list(map(int, r[1:])))
            expects.append([])
        elif r[0] == "expect":
            num, den = map(int, r[2].split("/"))
            expects[-1].append((int(r[1]), num, den, int(r[3], 16)))
    return bins, frame, np.array(boxes, np.int32), expects


def test_crop_hand_example(orc):
    bins, frame, boxes, expects = read_crop_golden()
    got = orc.hist_crops(frame, boxes, bins)
    for b, ex in enumerate(expects):
        want = np.zeros(bins ** 3, np.float32)
        for k, num, den, bits in ex:
            # the stated bits are the correctly rounded float32 of num/den
            assert (np.float32(num) / np.float32(den)).view(np.uint32) == bits
            want[k] = np.uint32(bits).view(np.float32)
        assert np.array_equal(got[b], want), "box %d" % b


def random_boxes(rng, nframes, height, width, m):
    f = rng.integers(0, nframes, size=m)
    x0 = rng.integers(0, width, size=m)
    y0 = rng.integers(0, height, size=m)
    x1 = x0 + 1 + rng.integers(0, width - x0)
    y1 = y0 + 1 + rng.integers(0, height - y0)
    return np.stack([f, x0, y0, x1, y1], axis=1).astype(np.int32)


@pytest.mark.parametrize("bins", [8, 4])
def test_crops_equal_histograms_of_sliced_patches(orc, bins):
    """A crop's histogram is the patch histogram of the cut-out pixels
    (numpy slicing, then the patch routine, itself pinned to histogramdd)."""
    rng = np.random.default_rng(31 + bins)
    frames = rng.integers(0, 256, size=(3, 23, 37, 3), dtype=np.uint8)
    boxes = random_boxes(rng, 3, 23, 37, 60)
    boxes[0] = (1, 0, 0, 37, 23)  # a whole frame
    boxes[1] = (2, 36, 22, 37, 23)  # the last pixel
    got = orc.hist_crops(frames, boxes, bins)
    for b, (f, x0, y0, x1, y1) in enumerate(boxes):
        patch = np.ascontiguousarray(frames[f, y0:y1, x0:x1][None])
        assert np.array_equal(got[b], orc.hist_rgb8(patch, bins)[0]), "box %d" % b


def test_crop_division_is_correctly_rounded(orc):
    """Pixel counts that are not powers of two: every bin is the IEEE single
    division count / area (correctly rounded), and the counts add up to the
    area."""
    rng = np.random.default_rng(5)
    frames = rng.integers(0, 256, size=(2, 31, 29, 3), dtype=np.uint8)
    boxes = random_boxes(rng, 2, 31, 29, 40)
    got = orc.hist_crops(frames, boxes, 8)
    for b, (f, x0, y0, x1, y1) in enumerate(boxes):
        area = (x1 - x0) * (y1 - y0)
        cnt = histogramdd_reference(np.ascontiguousarray(frames[f, y0:y1, x0:x1][None]), 8)[0]
        assert cnt.sum() == area
        assert np.array_equal(got[b], cnt.astype(np.float32) / np.float32(area))


def test_crop_outside_frame_is_rejected(orc):
    frames = np.zeros((2, 4, 5, 3), np.uint8)
    for bad in [(2, 0, 0, 1, 1), (0, 0, 0, 6, 1), (0, 3, 0, 3, 1), (0, 0, 2, 1, 5), (-1, 0, 0, 1, 1)]:
        with pytest.raises(ValueError):
            orc.hist_crops(frames, [bad], 8)
