"""Pins of the oracle's next operations (no GPU): reconstruction by erosion,
the h-dome and regional maxima.

* erosion against its defining iteration (exhaustive on tiny images, random
  at small sizes) and against the duality with reconstruction by dilation
  (the two are separate codes in the oracle);
* the h-dome against the defining iteration of the reconstruction it is made
  of, its bounds, and the closed form of an isolated peak;
* regional maxima against their definition, plateau by plateau through
  scipy.ndimage.label.
"""
import itertools

import numpy as np
import pytest

import brute
import synth


def _all_images(h, w, levels):
    vals = np.array(list(itertools.product(range(levels), repeat=h * w)), dtype=np.uint8)
    return vals.reshape(-1, h, w)


@pytest.mark.parametrize("conn", [4, 8])
def test_erosion_exhaustive_binary_3x3(oracle_mod, conn):
    imgs = _all_images(3, 3, 2) * 255
    for m in imgs[::7]:
        for k in imgs:
            assert np.array_equal(oracle_mod.recon_erode(m, k, conn), brute.iterate_erosion(m, k, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_erosion_random_against_definition(oracle_mod, conn):
    rng = np.random.default_rng(77 + conn)
    for h in range(1, 20, 3):
        for w in range(1, 20, 4):
            for levels in (2, 3, 256):
                for _ in range(6):
                    marker = rng.integers(0, levels, size=(h, w)).astype(np.uint8)
                    mask = rng.integers(0, levels, size=(h, w)).astype(np.uint8)
                    if levels == 256:
                        marker = np.clip(mask.astype(int) + rng.integers(1, 60), 0, 255).astype(np.uint8)
                    assert np.array_equal(oracle_mod.recon_erode(marker, mask, conn),
                                          brute.iterate_erosion(marker, mask, conn)), (h, w, levels)


@pytest.mark.parametrize("conn", [4, 8])
def test_erosion_duality(oracle_mod, conn):
    mask = synth.config1_tile()[1][:200, :300]
    rng = np.random.default_rng(5)
    for marker in (np.clip(mask.astype(int) + 25, 0, 255).astype(np.uint8),
                   rng.integers(0, 256, mask.shape).astype(np.uint8)):
        ero = oracle_mod.recon_erode(marker, mask, conn)
        dual = 255 - oracle_mod.recon_dilate(255 - marker, 255 - mask, conn)
        assert np.array_equal(ero, dual)
        assert (ero >= mask).all() and (ero <= np.maximum(marker, mask)).all()
        assert np.array_equal(oracle_mod.recon_erode(ero, mask, conn), ero)   # idempotent


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("h", [1, 7, 30])
def test_hdome_against_definition(oracle_mod, conn, h):
    rng = np.random.default_rng(h + conn)
    for _ in range(20):
        img = rng.integers(0, 256, size=(rng.integers(1, 18), rng.integers(1, 18))).astype(np.uint8)
        marker = np.clip(img.astype(int) - h, 0, 255).astype(np.uint8)
        want = img - brute.iterate_definition(marker, img, conn)
        got = oracle_mod.hdome(img, h, conn)
        assert np.array_equal(got, want)
        assert (got <= h).all()


def test_hdome_isolated_peak():
    """Background 40 with one pixel of 70: the marker max(I - h, 0) of the peak
    (70 - h) raises the background to min(70 - h, 40), so the dome is h at the
    peak and max(0, h - 30) on the background."""
    import oracle
    img = np.full((9, 9), 40, np.uint8)
    img[4, 4] = 70
    for h in (5, 30, 31, 45, 70):
        d = oracle.hdome(img, h, 8)
        want = np.full(img.shape, max(0, h - 30), np.uint8)
        want[4, 4] = h
        assert np.array_equal(d, want), h


@pytest.mark.parametrize("conn", [4, 8])
def test_regional_max_against_definition(oracle_mod, conn):
    rng = np.random.default_rng(100 + conn)
    for levels in (2, 3, 5, 256):
        for _ in range(15):
            img = rng.integers(0, levels, size=(rng.integers(1, 20), rng.integers(1, 20))).astype(np.uint8)
            if levels < 256:
                img = (img * (255 // (levels - 1))).astype(np.uint8)
            assert np.array_equal(oracle_mod.regional_max(img, conn), brute.regional_max_by_plateaus(img, conn))
    crop = synth.config1_tile()[1][:96, :96]
    assert np.array_equal(oracle_mod.regional_max(crop, conn), brute.regional_max_by_plateaus(crop, conn))


def test_regional_max_all_zero_reading(oracle_mod):
    assert not oracle_mod.regional_max(np.zeros((5, 7), np.uint8), 8).any()
