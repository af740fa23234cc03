"""GPU parity of the colour-histogram kernel against the oracle: bit-exact."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host
from paper_1812_07607_amd import ops, synth

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
