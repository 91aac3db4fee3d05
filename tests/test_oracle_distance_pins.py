"""Pins of the distance-transform and Pre-Watershed oracle (CPU only).

* brute force: the squared distance to every 0 pixel, minimised, on random
  small images (also with no 0 pixel at all);
* scipy.ndimage.distance_transform_edt (a library routine; its float
  distances squared and rounded are the exact integers) on the nuclei tiles;
* closed forms: one 0 pixel, all-zero, no zero, the 255 cap of D8;
* D8 against floor(sqrt) in float64 (exact for these magnitudes);
* the markers against regional maxima found plateau by plateau through
  scipy.ndimage.label (tests/brute.py), and on discs whose centre is known;
* planted mistakes in a copy of distance_oracle.c are each caught.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.ndimage as ndi

import brute
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "distance_oracle.c")
RECON_SRC = os.path.join(ROOT, "oracle", "recon_oracle.c")
CAP = 2 ** 31 - 1


def brute_distance2(img):
    zeros = np.argwhere(np.asarray(img) == 0)
    h, w = img.shape
    if len(zeros) == 0:
        return np.full((h, w), CAP, np.int64)
    yy, xx = np.mgrid[0:h, 0:w]
    d = (yy[..., None] - zeros[:, 0]) ** 2 + (xx[..., None] - zeros[:, 1]) ** 2
    return d.min(axis=-1)


def scipy_distance2(img):
    return np.rint(ndi.distance_transform_edt(np.asarray(img) != 0) ** 2).astype(np.int64)


def test_distance_brute_force(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(150):
        h, w = (int(v) for v in rng.integers(1, 30, 2))
        img = np.where(rng.random((h, w)) < rng.random() ** 0.3, 255, 0).astype(np.uint8)
        assert np.array_equal(oracle_mod.distance2(img), brute_distance2(img))


def test_distance_equals_scipy(oracle_mod):
    _, _, binary = synth.config2_tile(seed=synth.seed_for(2, 41), size=1024, n_gauss=188)
    assert np.array_equal(oracle_mod.distance2(binary), scipy_distance2(binary))
    rng = np.random.default_rng(2)
    for p in (0.5, 0.9, 0.999):
        img = np.where(rng.random((300, 517)) < p, 255, 0).astype(np.uint8)
        assert np.array_equal(oracle_mod.distance2(img), scipy_distance2(img))


def test_distance_closed_forms(oracle_mod):
    img = np.full((40, 70), 9, np.uint8)
    img[13, 50] = 0
    yy, xx = np.mgrid[0:40, 0:70]
    assert np.array_equal(oracle_mod.distance2(img), (yy - 13) ** 2 + (xx - 50) ** 2)
    assert not oracle_mod.distance2(np.zeros((5, 6), np.uint8)).any()
    assert (oracle_mod.distance2(np.full((5, 6), 1, np.uint8)) == CAP).all()
    assert (oracle_mod.distance8(np.full((5, 6), 1, np.uint8)) == 255).all()
    # the cap of D8: a corner 0 pixel in a 400 x 400 image
    big = np.full((400, 400), 255, np.uint8)
    big[0, 0] = 0
    yy, xx = np.mgrid[0:400, 0:400]
    want = np.minimum(np.floor(np.sqrt((yy ** 2 + xx ** 2).astype(np.float64))), 255).astype(np.uint8)
    assert np.array_equal(oracle_mod.distance8(big), want)
    assert oracle_mod.distance8(big)[399, 399] == 255 and oracle_mod.distance8(big)[0, 255] == 255
    assert oracle_mod.distance8(big)[0, 254] == 254


def test_distance8_is_floor_sqrt(oracle_mod):
    _, _, binary = synth.config2_tile(seed=synth.seed_for(2, 42), size=512, n_gauss=47)
    d2 = oracle_mod.distance2(binary).astype(np.float64)
    want = np.minimum(np.floor(np.sqrt(d2)), 255).astype(np.uint8)
    assert np.array_equal(oracle_mod.distance8(binary), want)


@pytest.mark.parametrize("conn", [4, 8])
def test_markers_are_regional_maxima_of_d8(oracle_mod, conn):
    _, _, binary = synth.config2_tile(seed=synth.seed_for(2, 43), size=384, n_gauss=27)
    d8 = oracle_mod.distance8(binary)
    assert np.array_equal(oracle_mod.pre_watershed(binary, conn), brute.regional_max_by_plateaus(d8, conn))


def test_markers_of_discs(oracle_mod):
    # two discs of radius 9 centred on pixels: each has one marker, at its centre
    yy, xx = np.mgrid[0:60, 0:90]
    img = np.zeros((60, 90), np.uint8)
    for cy, cx in ((20, 25), (35, 65)):
        img[(yy - cy) ** 2 + (xx - cx) ** 2 <= 81] = 255
    for conn in (4, 8):
        m = oracle_mod.pre_watershed(img, conn)
        assert sorted(map(tuple, np.argwhere(m > 0))) == [(20, 25), (35, 65)]


MUTANTS = {
    "no_up_scan": ("if (d != none && (g[y * w + x] == none || d < g[y * w + x])) g[y * w + x] = d;", "(void)0;"),
    "left_only": ("if (step == 0 && side == 1) break;", "if (side == 1) break;"),
    "isqrt_low": ("while ((r + 1) * (r + 1) <= v) ++r;", "while ((r + 1) * (r + 1) < v) ++r;"),
    "outside_is_background": ("int64_t d = none;\n        for (int64_t y = 0; y < h; ++y) {",
                              "int64_t d = 0;\n        for (int64_t y = 0; y < h; ++y) {"),
    "markers_conn4": ("if (rc == 0) rc = oracle_regional_max(d8, out, h, w, conn);",
                      "if (rc == 0) rc = oracle_regional_max(d8, out, h, w, 4);"),
}


def _lib(tmp_path, name=None):
    src = open(SRC).read()
    if name:
        old, new = MUTANTS[name]
        assert src.count(old) == 1, "mutation site for %s not unique" % name
        src = src.replace(old, new)
    path = tmp_path / ("d_%s.c" % (name or "plain"))
    path.write_text(src)
    so = tmp_path / ("d_%s.so" % (name or "plain"))
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(path), RECON_SRC], check=True)
    lib = ctypes.CDLL(str(so))
    lib.oracle_distance2.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2
    lib.oracle_distance8.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2
    lib.oracle_pre_watershed.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_int]
    return lib


def _pins_pass(lib):
    rng = np.random.default_rng(5)
    for _ in range(30):
        h, w = (int(v) for v in rng.integers(2, 25, 2))
        img = np.where(rng.random((h, w)) < 0.8, 255, 0).astype(np.uint8)
        d2 = np.empty((h, w), np.int32)
        lib.oracle_distance2(img.ctypes.data, d2.ctypes.data, h, w)
        if not np.array_equal(d2, brute_distance2(img)):
            return False
        d8 = np.empty((h, w), np.uint8)
        lib.oracle_distance8(img.ctypes.data, d8.ctypes.data, h, w)
        want8 = np.minimum(np.floor(np.sqrt(brute_distance2(img).astype(np.float64))), 255).astype(np.uint8)
        if not np.array_equal(d8, want8):
            return False
    _, _, binary = synth.config2_tile(seed=synth.seed_for(2, 44), size=256, n_gauss=12)
    for conn in (4, 8):
        m = np.empty_like(binary)
        lib.oracle_pre_watershed(binary.ctypes.data, m.ctypes.data, 256, 256, conn)
        d8 = np.minimum(np.floor(np.sqrt(scipy_distance2(binary).astype(np.float64))), 255).astype(np.uint8)
        if not np.array_equal(m, brute.regional_max_by_plateaus(d8, conn)):
            return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_lib(tmp_path, name)), "planted mistake %s passed every pin" % name


def test_unmutated_source_passes(tmp_path):
    assert _pins_pass(_lib(tmp_path))
