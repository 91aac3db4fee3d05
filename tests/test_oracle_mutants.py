"""Planted mistakes in a copy of the oracle must be caught by the pins (CPU only).

Each mutant is the oracle's C source with one plausible slip (a dropped
neighbour, a missing mask cap, a wrong comparison, a wrong frame) compiled into a
temporary library.  (Dropping the initial clip is not listed: the raster
scan caps every pixel by the mask before any later pixel reads it, so that
mutant is equivalent.)  The test runs the same pins as test_oracle_pins.py on a
small budget and requires at least one of them to fail for every mutant, so
that the pins are shown to have teeth.  The real oracle is never modified.
"""
import ctypes
import itertools
import os
import subprocess

import numpy as np
import pytest

import brute

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "recon_oracle.c")

MUTANTS = {
    "raster_drops_NE": ("{-1, 0}, {-1, 1}};\nstatic const int LATE8", "{-1, 0}, {-1, 0}};\nstatic const int LATE8"),
    "late_drops_SW": ("{1, 0}, {1, -1}};", "{1, 0}, {1, 0}};"),
    "anti_raster_mask_cap": ("J[p] = u8min(m, I[p]);", "J[p] = m;"),
    "fifo_ignores_mask": ("J[r] = u8min(J[p], I[r]);", "J[r] = J[p];"),
    "seed_test_wrong_side": ("if (J[r] < J[p] && J[r] < I[r]) {", "if (J[r] > J[p] && J[r] < I[r]) {"),
    "no_fifo_push": ("J[r] = u8min(J[p], I[r]);\n                    if (fifo_push(&q, r) != 0) { free(q.buf); return -2; }",
                     "J[r] = u8min(J[p], I[r]);\n                    (void)0;"),
    "raster_mask_cap": ("J[y * w + x] = u8min(m, I[y * w + x]);", "J[y * w + x] = m;"),
    "fill_frame_rows_only": ("y == 0 || y == height - 1 || x == 0 || x == width - 1",
                             "y == 0 || y == height - 1"),
    "fill_not_complemented": ("out[i] = (uint8_t)(255 - out[i]);", "(void)0;"),
    # reconstruction by erosion, h-dome, regional maxima
    "erode_raster_floor": ("J[y * w + x] = u8max(m, I[y * w + x]);", "J[y * w + x] = m;"),
    "erode_fifo_floor": ("J[r] = u8max(J[p], I[r]);", "J[r] = J[p];"),
    "erode_seed_wrong_side": ("if (J[r] > J[p] && J[r] > I[r]) {", "if (J[r] < J[p] && J[r] > I[r]) {"),
    "erode_no_fifo_push": ("J[r] = u8max(J[p], I[r]);\n                    if (fifo_push(&q, r) != 0) { free(q.buf); return -2; }",
                           "J[r] = u8max(J[p], I[r]);\n                    (void)0;"),
    "hdome_marker_off_by_one": ("img[i] > hval ? img[i] - hval : 0", "img[i] > hval ? img[i] - hval + 1 : 0"),
    "rmax_threshold": ("out[i] = out[i] ? 255 : 0;", "out[i] = out[i] > 1 ? 255 : 0;"),
}


def _build_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site for %s not unique" % name
    path = tmp_path / ("m_%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("m_%s.so" % name)
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(path)],
                   check=True)
    lib = ctypes.CDLL(str(so))
    _declare(lib)
    return lib


def _declare(lib):
    lib.oracle_recon_dilate_many.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64] * 3 + [ctypes.c_int]
    lib.oracle_fill_holes.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_int]
    lib.oracle_recon_erode.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64] * 2 + [ctypes.c_int]
    lib.oracle_hdome.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_int, ctypes.c_int]
    lib.oracle_regional_max.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_int]


def _pins_pass(lib):
    """True if the mutant passes every pin in this small budget."""
    # exhaustive 3-level 2x3 and binary 3x3 against the defining iteration
    for (h, w, levels) in [(2, 3, 3), (3, 3, 2), (1, 4, 3)]:
        imgs = np.array(list(itertools.product(range(levels), repeat=h * w)), np.uint8).reshape(-1, h, w)
        if levels == 2:
            imgs = imgs * 255
        n = len(imgs)
        markers = np.ascontiguousarray(np.repeat(imgs, n, axis=0))
        masks = np.ascontiguousarray(np.tile(imgs, (n, 1, 1)))
        for conn in (4, 8):
            out = np.empty_like(markers)
            rc = lib.oracle_recon_dilate_many(markers.ctypes.data, masks.ctypes.data, out.ctypes.data,
                                              len(markers), h, w, conn)
            if rc != 0 or not np.array_equal(out, brute.iterate_definition(markers, masks, conn)):
                return False
    rng = np.random.default_rng(3)
    for conn in (4, 8):
        for _ in range(20):
            x = np.where(rng.random((9, 11)) < 0.5, 255, 0).astype(np.uint8)
            out = np.empty_like(x)
            lib.oracle_fill_holes(x.ctypes.data, out.ctypes.data, 9, 11, conn)
            if not np.array_equal(out, brute.fill_holes_binary(x, conn)):
                return False
    # reconstruction by erosion, h-dome and regional maxima against their definitions
    for conn in (4, 8):
        for _ in range(30):
            h, w = rng.integers(1, 9, size=2)
            mask = rng.integers(0, 4, size=(h, w)).astype(np.uint8) * 60
            marker = np.clip(mask.astype(int) + rng.integers(0, 200, size=(h, w)), 0, 255).astype(np.uint8)
            out = np.empty_like(mask)
            lib.oracle_recon_erode(marker.ctypes.data, mask.ctypes.data, out.ctypes.data, h, w, conn)
            if not np.array_equal(out, brute.iterate_erosion(marker, mask, conn)):
                return False
            img = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
            lib.oracle_hdome(img.ctypes.data, out.ctypes.data, h, w, 9, conn)
            want = img - brute.iterate_definition(np.clip(img.astype(int) - 9, 0, 255).astype(np.uint8), img, conn)
            if not np.array_equal(out, want):
                return False
            lib.oracle_regional_max(img.ctypes.data, out.ctypes.data, h, w, conn)
            if not np.array_equal(out, brute.regional_max_by_plateaus(img, conn)):
                return False
    return True


def test_unmutated_copy_passes(tmp_path):
    src = open(SRC).read()
    path = tmp_path / "same.c"
    path.write_text(src)
    so = tmp_path / "same.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(path)], check=True)
    lib = ctypes.CDLL(str(so))
    _declare(lib)
    assert _pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_build_mutant(tmp_path, name)), "pins missed mutant %s" % name
