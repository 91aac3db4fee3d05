"""Properties of the synthetic input generators (no GPU, no oracle arithmetic)."""
import numpy as np
import scipy.ndimage as ndi

import synth


def test_config1_shape_and_determinism():
    m1, i1 = synth.config1_tile()
    m2, i2 = synth.config1_tile()
    assert i1.shape == (512, 512) and i1.dtype == np.uint8
    assert np.array_equal(i1, i2) and np.array_equal(m1, m2)
    assert np.array_equal(m1, np.clip(i1.astype(int) - 30, 0, 255))
    assert i1.max() > 100  # blobs present


def test_config2_small_density():
    marker, mask, binary = synth.config2_tile(seed=synth.seed_for(2, 1), size=256, n_gauss=12)
    assert mask.shape == (256, 256)
    assert set(np.unique(binary)) <= {0, 255}
    assert np.array_equal(binary > 0, mask > 120)
    # background 30 with noise [-10, 10]: nothing below 20
    assert mask.min() >= 20


def test_spiral_is_one_chain():
    for (h, w) in [(4, 4), (5, 9), (64, 64), (257, 131), (512, 512)]:
        path = synth.spiral_path(h, w)
        assert len(np.unique(path[:, 0] * w + path[:, 1])) == len(path)
        steps = np.abs(np.diff(path, axis=0)).sum(1)
        assert np.all(steps == 1)  # consecutive cells are edge neighbours
        marker, mask, n = synth.spiral_tile(h, w, "inner")
        for c in (1, 2):
            _, k = ndi.label(mask > 0, structure=ndi.generate_binary_structure(2, c))
            assert k == 1
        assert marker.sum() == 255 and n == len(path)
        # a large share of the tile is corridor
        assert n >= 0.4 * h * w


def test_config4_shapes():
    shapes = synth.config4_shapes()
    assert len(shapes) == 256
    for h, w, c, hv in shapes:
        assert h in synth.SIZES_CFG4 and w in synth.SIZES_CFG4
        assert c in (4, 8) and 10 <= hv <= 40
    conns = [s[2] for s in shapes]
    assert 80 < conns.count(4) < 176
