"""Pins of the labelling and area-filter oracle (BWLabel, AreaThreshold of the
paper's Table 1), CPU only.

* scipy.ndimage.label (a library routine; it numbers components in the same
  raster order of first pixels) on random images of every density and on the
  binary nuclei tile;
* the defining propagation (tests/brute.py), exhaustively on every binary 3x3
  and 2x4 / 4x2 image, and on random small images;
* closed forms: empty, full, checkerboards, diagonal lines, the spiral
  corridor (one component under both connectivities);
* the area filter against label counts through numpy, and its closed forms;
* planted mistakes in a copy of label_oracle.c are each caught.
"""
import ctypes
import itertools
import os
import subprocess

import numpy as np
import pytest
import scipy.ndimage as ndi

import brute
import synth

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "label_oracle.c")


def _scipy_label(img, conn):
    return ndi.label(np.asarray(img) != 0, structure=ndi.generate_binary_structure(2, 1 if conn == 4 else 2))


@pytest.mark.parametrize("conn", [4, 8])
def test_label_equals_scipy(oracle_mod, conn):
    rng = np.random.default_rng(100 + conn)
    for _ in range(150):
        h, w = (int(v) for v in rng.integers(1, 90, 2))
        img = np.where(rng.random((h, w)) < rng.random(), 255, 0).astype(np.uint8)
        lab, n = oracle_mod.label(img, conn)
        want, wn = _scipy_label(img, conn)
        assert n == wn and np.array_equal(lab, want)
    # grey input: every nonzero pixel is foreground
    img = rng.integers(0, 3, (64, 300)).astype(np.uint8)
    lab, n = oracle_mod.label(img, conn)
    want, wn = _scipy_label(img, conn)
    assert n == wn and np.array_equal(lab, want)


def test_label_nuclei_tile_equals_scipy(oracle_mod):
    _, mask, binary = synth.config2_tile(seed=synth.seed_for(2, 31), size=1024, n_gauss=188)
    for conn in (4, 8):
        lab, n = oracle_mod.label(binary, conn)
        want, wn = _scipy_label(binary, conn)
        assert n == wn and n > 50 and np.array_equal(lab, want)


@pytest.mark.parametrize("shape", [(3, 3), (2, 4), (4, 2), (1, 6)])
def test_label_exhaustive_against_propagation(oracle_mod, shape):
    h, w = shape
    for bits in itertools.product((0, 255), repeat=h * w):
        img = np.array(bits, np.uint8).reshape(h, w)
        for conn in (4, 8):
            lab, n = oracle_mod.label(img, conn)
            want, wn = brute.label_by_propagation(img, conn)
            assert n == wn and np.array_equal(lab, want), (img.tolist(), conn)


def test_label_random_against_propagation(oracle_mod):
    rng = np.random.default_rng(7)
    for _ in range(60):
        h, w = (int(v) for v in rng.integers(1, 30, 2))
        img = np.where(rng.random((h, w)) < 0.55, 255, 0).astype(np.uint8)
        for conn in (4, 8):
            lab, n = oracle_mod.label(img, conn)
            want, wn = brute.label_by_propagation(img, conn)
            assert n == wn and np.array_equal(lab, want)


def test_label_closed_forms(oracle_mod):
    for conn in (4, 8):
        z = np.zeros((7, 9), np.uint8)
        lab, n = oracle_mod.label(z, conn)
        assert n == 0 and not lab.any()
        lab, n = oracle_mod.label(np.full((7, 9), 3, np.uint8), conn)
        assert n == 1 and (lab == 1).all()
    # checkerboard: every foreground pixel alone under 4-connectivity, one component under 8
    yy, xx = np.mgrid[0:6, 0:8]
    cb = np.where((yy + xx) % 2 == 0, 255, 0).astype(np.uint8)
    lab, n = oracle_mod.label(cb, 4)
    assert n == int((cb > 0).sum())
    order = np.flatnonzero(cb.ravel())                  # raster order of the single pixels
    assert np.array_equal(lab.ravel()[order], np.arange(1, n + 1))
    lab, n = oracle_mod.label(cb, 8)
    assert n == 1
    # an anti-diagonal line: n pixels under 4, one component under 8; numbering by first pixel
    d = np.fliplr(np.eye(5, dtype=np.uint8) * 255)
    lab, n = oracle_mod.label(d, 4)
    assert n == 5 and lab[0, 4] == 1 and lab[4, 0] == 5
    lab, n = oracle_mod.label(d, 8)
    assert n == 1
    # the spiral corridor is one component under both connectivities
    _, corridor, _ = synth.spiral_tile(64, 96, "outer")
    for conn in (4, 8):
        lab, n = oracle_mod.label(corridor, conn)
        assert n == 1 and np.array_equal(lab > 0, corridor > 0)


@pytest.mark.parametrize("conn", [4, 8])
def test_area_threshold_equals_counts(oracle_mod, conn):
    rng = np.random.default_rng(200 + conn)
    for _ in range(60):
        h, w = (int(v) for v in rng.integers(1, 70, 2))
        img = np.where(rng.random((h, w)) < rng.random(), 255, 0).astype(np.uint8)
        lo, hi = sorted(int(v) for v in rng.integers(0, 40, 2))
        lab, n = _scipy_label(img, conn)
        area = np.bincount(lab.ravel(), minlength=n + 1)
        keep = (area >= lo) & (area <= hi)
        keep[0] = False
        want = np.where(keep[lab], 255, 0).astype(np.uint8)
        assert np.array_equal(oracle_mod.area_threshold(img, lo, hi, conn), want), (lo, hi)


def test_area_threshold_closed_forms(oracle_mod):
    img = np.zeros((10, 12), np.uint8)
    img[1:3, 1:4] = 255      # area 6
    img[5, 5] = 255          # area 1
    img[7:10, 8:12] = 9      # area 12
    both = np.where(img > 0, 255, 0).astype(np.uint8)
    for conn in (4, 8):
        assert np.array_equal(oracle_mod.area_threshold(img, 1, 1 << 40, conn), both)
        assert not oracle_mod.area_threshold(img, 13, 100, conn).any()
        only6 = oracle_mod.area_threshold(img, 6, 6, conn)            # bounds are inclusive
        assert np.array_equal(only6 > 0, np.pad(np.ones((2, 3), bool), ((1, 7), (1, 8))))
        single = np.zeros_like(both, bool)
        single[5, 5] = True
        assert np.array_equal(oracle_mod.area_threshold(img, 2, 12, conn) > 0, (img > 0) & ~single)


# ---- planted mistakes

MUTANTS = {
    "conn8_drops_corners": ("const int *dy = conn == 8 ? dy8 : dy4, *dx = conn == 8 ? dx8 : dx4;",
                            "const int *dy = dy4, *dx = dx4; conn = 4;"),
    "bounds_off_by_one": ("if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;",
                          "if (yy < 0 || yy >= h || xx < 0 || xx > w) continue;"),
    "labels_from_zero": ("labels[s] = ++next;", "labels[s] = next++ + 1; labels[s] -= 1;"),
    "grey_is_background": ("if (img[s] == 0 || labels[s] != 0) continue;",
                           "if (img[s] != 255 || labels[s] != 0) continue;"),
    "area_min_exclusive": ("out[p] = (l != 0 && area[l] >= min_area", "out[p] = (l != 0 && area[l] > min_area"),
    "area_keeps_background": ("out[p] = (l != 0 && area[l] >= min_area", "out[p] = (area[l] >= min_area"),
}


def _mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site for %s not unique" % name
    path = tmp_path / ("m_%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("m_%s.so" % name)
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(path)], check=True)
    lib = ctypes.CDLL(str(so))
    lib.oracle_label.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_int]
    lib.oracle_label.restype = ctypes.c_int64
    lib.oracle_area_threshold.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_int] + \
        [ctypes.c_int64] * 2
    lib.oracle_area_threshold.restype = ctypes.c_int64
    return lib


def _pins_pass(lib):
    rng = np.random.default_rng(3)
    for _ in range(40):
        h, w = (int(v) for v in rng.integers(1, 20, 2))
        img = np.where(rng.random((h, w)) < 0.5, 255, rng.integers(0, 2, (h, w))).astype(np.uint8)
        for conn in (4, 8):
            lab = np.empty((h, w), np.int32)
            n = lib.oracle_label(img.ctypes.data, lab.ctypes.data, h, w, conn)
            want, wn = _scipy_label(img, conn)
            if n != wn or not np.array_equal(lab, want):
                return False
            lo, hi = 2, 9
            out = np.empty((h, w), np.uint8)
            lib.oracle_area_threshold(img.ctypes.data, out.ctypes.data, h, w, conn, lo, hi)
            area = np.bincount(want.ravel(), minlength=wn + 1)
            keep = (area >= lo) & (area <= hi)
            keep[0] = False
            if not np.array_equal(out, np.where(keep[want], 255, 0).astype(np.uint8)):
                return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_mutant(tmp_path, name)), "planted mistake %s passed every pin" % name


def test_unmutated_source_passes(tmp_path):
    so = tmp_path / "plain.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), SRC], check=True)
    lib = ctypes.CDLL(str(so))
    lib.oracle_label.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_int]
    lib.oracle_label.restype = ctypes.c_int64
    lib.oracle_area_threshold.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_int] + \
        [ctypes.c_int64] * 2
    lib.oracle_area_threshold.restype = ctypes.c_int64
    assert _pins_pass(lib)
