"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

The oracle (Vincent's hybrid sequential algorithm) is checked against
  * hand-worked fixtures (tests/golden),
  * the defining iteration, exhaustively on tiny images and at random,
  * threshold decomposition through a library labelling at realistic sizes,
  * scipy's binary fill-holes (binary and level-by-level grey),
  * closed forms (single rows, constant masks, spiral corridors),
  * invariants (bounds, idempotence, monotonicity, stability, h-dome bound).
"""
import itertools

import numpy as np
import pytest

import brute
import golden_io
import synth


# ---- hand-worked fixtures -----------------------------------------------------

@pytest.mark.parametrize("case", golden_io.all_cases(), ids=lambda c: c["name"])
def test_golden(oracle_mod, case):
    for conn in case["conns"]:
        if case["op"] == "dilate":
            got = oracle_mod.recon_dilate(case["marker"], case["mask"], conn)
        else:
            got = oracle_mod.fill_holes(case["img"], conn)
        np.testing.assert_array_equal(got, case["expect"], err_msg="conn=%d" % conn)


# ---- exhaustive tiny images against the defining iteration ----------------------

def _all_images(h, w, levels):
    vals = np.array(list(itertools.product(range(levels), repeat=h * w)), dtype=np.uint8)
    return vals.reshape(-1, h, w)


@pytest.mark.parametrize("conn", [4, 8])
def test_exhaustive_binary_3x3(oracle_mod, conn):
    imgs = _all_images(3, 3, 2) * 255
    n = len(imgs)
    markers = np.repeat(imgs, n, axis=0)
    masks = np.tile(imgs, (n, 1, 1))
    got = oracle_mod.recon_dilate_many(markers, masks, conn)
    want = brute.iterate_definition(markers, masks, conn)
    bad = np.nonzero((got != want).reshape(len(got), -1).any(1))[0]
    assert bad.size == 0, "first mismatch at case %d" % (bad[0] if bad.size else -1)


@pytest.mark.parametrize("shape", [(2, 2), (1, 4), (4, 1), (2, 3), (3, 2)])
@pytest.mark.parametrize("conn", [4, 8])
def test_exhaustive_three_levels(oracle_mod, shape, conn):
    imgs = _all_images(shape[0], shape[1], 3)
    n = len(imgs)
    markers = np.repeat(imgs, n, axis=0)
    masks = np.tile(imgs, (n, 1, 1))
    got = oracle_mod.recon_dilate_many(markers, masks, conn)
    want = brute.iterate_definition(markers, masks, conn)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("conn", [4, 8])
def test_random_small_against_definition(oracle_mod, conn):
    rng = np.random.default_rng(1234 + conn)
    for h in range(1, 25, 3):
        for w in range(1, 25, 4):
            for levels in (2, 3, 5, 256):
                markers = rng.integers(0, levels, size=(40, h, w)).astype(np.uint8)
                masks = rng.integers(0, levels, size=(40, h, w)).astype(np.uint8)
                if levels == 256:
                    # h-dome style markers: the shape used by the workloads
                    markers[:20] = np.clip(masks[:20].astype(int) - rng.integers(1, 60), 0, 255)
                got = oracle_mod.recon_dilate_many(markers, masks, conn)
                want = brute.iterate_definition(markers, masks, conn)
                assert np.array_equal(got, want), (h, w, levels)


# ---- library pins at realistic sizes ------------------------------------------------

@pytest.mark.parametrize("conn", [4, 8])
def test_threshold_decomposition_config1(oracle_mod, conn):
    marker, mask = synth.config1_tile()
    got = oracle_mod.recon_dilate(marker, mask, conn)
    want = brute.threshold_decomposition(marker, mask, conn)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("conn", [4, 8])
def test_threshold_decomposition_nuclei_crop(oracle_mod, conn):
    # config-2 density on a 384 x 384 crop (same generator, 3000 * (384/4096)^2 Gaussians)
    marker, mask, _ = synth.config2_tile(seed=synth.seed_for(2, 17), size=384, n_gauss=26)
    got = oracle_mod.recon_dilate(marker, mask, conn)
    want = brute.threshold_decomposition(marker, mask, conn)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("conn", [4, 8])
def test_fill_holes_binary_library(oracle_mod, conn):
    rng = np.random.default_rng(77 + conn)
    for (h, w) in [(1, 1), (1, 7), (7, 1), (2, 2), (3, 3), (5, 9), (31, 17), (64, 64)]:
        for p in (0.3, 0.5, 0.7):
            x = np.where(rng.random((h, w)) < p, 255, 0).astype(np.uint8)
            assert np.array_equal(oracle_mod.fill_holes(x, conn), brute.fill_holes_binary(x, conn))
    _, _, binary = synth.config2_tile(seed=synth.seed_for(2, 3), size=512, n_gauss=47)
    assert np.array_equal(oracle_mod.fill_holes(binary, conn), brute.fill_holes_binary(binary, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_fill_holes_grey_by_levels(oracle_mod, conn):
    rng = np.random.default_rng(99 + conn)
    for (h, w) in [(1, 5), (4, 4), (9, 13), (24, 24)]:
        for levels in (3, 8, 256):
            x = rng.integers(0, levels, size=(h, w)).astype(np.uint8)
            assert np.array_equal(oracle_mod.fill_holes(x, conn), brute.fill_holes_by_levels(x, conn))
    # a grey nuclei-like crop
    _, mask, _ = synth.config2_tile(seed=synth.seed_for(2, 5), size=96, n_gauss=2)
    assert np.array_equal(oracle_mod.fill_holes(mask, conn), brute.fill_holes_by_levels(mask, conn))


# ---- closed forms --------------------------------------------------------------------

@pytest.mark.parametrize("conn", [4, 8])
def test_single_row_and_column(oracle_mod, conn):
    rng = np.random.default_rng(5)
    for n in (1, 2, 3, 17, 300):
        for levels in (3, 256):
            mask = rng.integers(0, levels, size=n).astype(np.uint8)
            marker = rng.integers(0, levels, size=n).astype(np.uint8)
            want = brute.row_closed_form(marker, mask)
            assert np.array_equal(oracle_mod.recon_dilate(marker[None], mask[None], conn)[0], want)
            assert np.array_equal(oracle_mod.recon_dilate(marker[:, None], mask[:, None], conn)[:, 0], want)


@pytest.mark.parametrize("conn", [4, 8])
def test_constant_mask(oracle_mod, conn):
    rng = np.random.default_rng(6)
    for c in (0, 1, 128, 255):
        mask = np.full((37, 53), c, np.uint8)
        marker = rng.integers(0, 256, size=mask.shape).astype(np.uint8)
        got = oracle_mod.recon_dilate(marker, mask, conn)
        assert np.all(got == min(int(marker.max()), c))


@pytest.mark.parametrize("seed_at", ["outer", "inner"])
@pytest.mark.parametrize("conn", [4, 8])
def test_spiral_fills_corridor(oracle_mod, seed_at, conn):
    marker, mask, n = synth.spiral_tile(257, 131, seed_at)
    got = oracle_mod.recon_dilate(marker, mask, conn)
    assert np.array_equal(got, mask)
    # against the definition too (short enough here)
    assert np.array_equal(got, brute.iterate_definition(marker, mask, conn))


# ---- invariants ----------------------------------------------------------------------

@pytest.mark.parametrize("conn", [4, 8])
def test_invariants(oracle_mod, conn):
    rng = np.random.default_rng(11 + conn)
    for trial in range(30):
        h, w = rng.integers(1, 40, size=2)
        levels = [2, 4, 16, 256][trial % 4]
        marker, mask = synth.random_pair(rng, h, w, levels)
        rho = oracle_mod.recon_dilate(marker, mask, conn)
        assert np.all(rho >= np.minimum(marker, mask)) and np.all(rho <= mask)
        assert np.array_equal(oracle_mod.recon_dilate(rho, mask, conn), rho)  # idempotent
        assert np.array_equal(np.minimum(brute.dilate(rho, conn), mask), rho)  # stable
        assert np.array_equal(oracle_mod.recon_dilate(mask, mask, conn), mask)
        assert not oracle_mod.recon_dilate(np.zeros_like(mask), mask, conn).any()
        # monotone in the marker and in the mask
        bigger_marker = np.maximum(marker, rng.integers(0, levels, size=(h, w)).astype(np.uint8))
        assert np.all(oracle_mod.recon_dilate(bigger_marker, mask, conn) >= rho)
        bigger_mask = np.maximum(mask, rng.integers(0, levels, size=(h, w)).astype(np.uint8))
        assert np.all(oracle_mod.recon_dilate(marker, bigger_mask, conn) >= rho)
        # h-dome bound
        hv = int(rng.integers(1, 50))
        dome = mask.astype(int) - oracle_mod.recon_dilate(synth.hdome_marker(mask, hv), mask, conn)
        assert dome.min() >= 0 and dome.max() <= hv


def test_fill_holes_frame_unchanged_and_extensive(oracle_mod):
    rng = np.random.default_rng(21)
    for _ in range(20):
        h, w = rng.integers(1, 30, size=2)
        x = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
        for conn in (4, 8):
            f = oracle_mod.fill_holes(x, conn)
            assert np.all(f >= x)
            assert np.array_equal(f[0], x[0]) and np.array_equal(f[-1], x[-1])
            assert np.array_equal(f[:, 0], x[:, 0]) and np.array_equal(f[:, -1], x[:, -1])
            assert np.array_equal(oracle_mod.fill_holes(f, conn), f)


def test_argument_errors(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.recon_dilate(np.zeros((2, 2), np.uint8), np.zeros((2, 3), np.uint8), 8)
    with pytest.raises(ValueError):
        oracle_mod.recon_dilate(np.zeros((2, 2), np.uint8), np.zeros((2, 2), np.uint8), 6)
    with pytest.raises(TypeError):
        oracle_mod.recon_dilate(np.zeros((2, 2), np.int32), np.zeros((2, 2), np.uint8), 8)
