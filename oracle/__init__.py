"""CPU oracle for grayscale reconstruction by dilation and fill-holes, the
operations built on it (erosion, h-dome, regional maxima), and connected-
component labelling with the area filter, and the exact distance transform
with the Pre-Watershed markers.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``.  The product library never
imports, links or runs anything in this directory.

The arithmetic lives in ``recon_oracle.c``, ``label_oracle.c`` and
``distance_oracle.c`` (plain C, built with gcc); this module only compiles
them and marshals numpy arrays through ctypes.  See those files' headers for the definitions followed (the
Table 1 operations of Sec. V-A) and for the sequential algorithms.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "recon_oracle.c"), os.path.join(_HERE, "label_oracle.c"),
         os.path.join(_HERE, "distance_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        # -O3; x86-64-v3 (AVX2) rather than -march=native, because the library may be
        # built on one machine and loaded on another whose CPU lacks newer extensions
        subprocess.run(["gcc", "-O3", "-march=x86-64-v3", "-std=c99", "-fPIC", "-shared", "-o", tmp] + _SRCS,
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_recon_dilate.argtypes = [u8p, u8p, u8p, i64, i64, ctypes.c_int]
        lib.oracle_recon_dilate.restype = ctypes.c_int
        lib.oracle_fill_holes.argtypes = [u8p, u8p, i64, i64, ctypes.c_int]
        lib.oracle_fill_holes.restype = ctypes.c_int
        lib.oracle_recon_dilate_many.argtypes = [u8p, u8p, u8p, i64, i64, i64, ctypes.c_int]
        lib.oracle_recon_dilate_many.restype = ctypes.c_int
        lib.oracle_recon_erode.argtypes = [u8p, u8p, u8p, i64, i64, ctypes.c_int]
        lib.oracle_recon_erode.restype = ctypes.c_int
        lib.oracle_hdome.argtypes = [u8p, u8p, i64, i64, ctypes.c_int, ctypes.c_int]
        lib.oracle_hdome.restype = ctypes.c_int
        lib.oracle_regional_max.argtypes = [u8p, u8p, i64, i64, ctypes.c_int]
        lib.oracle_regional_max.restype = ctypes.c_int
        lib.oracle_label.argtypes = [u8p, u8p, i64, i64, ctypes.c_int]
        lib.oracle_label.restype = i64
        lib.oracle_area_threshold.argtypes = [u8p, u8p, i64, i64, ctypes.c_int, i64, i64]
        lib.oracle_area_threshold.restype = i64
        for name in ("oracle_distance2", "oracle_distance8"):
            getattr(lib, name).argtypes = [u8p, u8p, i64, i64]
            getattr(lib, name).restype = ctypes.c_int
        lib.oracle_pre_watershed.argtypes = [u8p, u8p, i64, i64, ctypes.c_int]
        lib.oracle_pre_watershed.restype = ctypes.c_int
        _lib = lib
    return _lib


def _u8(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint8:
        raise TypeError("oracle images are uint8, got %s" % a.dtype)
    return a


def recon_dilate(marker, mask, conn: int = 8) -> np.ndarray:
    """rho_mask(marker): reconstruction by dilation (marker clipped under mask)."""
    marker, mask = _u8(marker), _u8(mask)
    if marker.shape != mask.shape or marker.ndim != 2:
        raise ValueError("marker and mask must be 2-D arrays of one shape")
    out = np.empty_like(marker)
    h, w = marker.shape
    rc = _load().oracle_recon_dilate(marker.ctypes.data, mask.ctypes.data, out.ctypes.data,
                                     h, w, int(conn))
    if rc != 0:
        raise ValueError("oracle_recon_dilate failed with %d" % rc)
    return out


def fill_holes(img, conn: int = 8) -> np.ndarray:
    """255 - rho_{255-img}(frame marker): fill-holes as reconstruction of the complement."""
    img = _u8(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    out = np.empty_like(img)
    h, w = img.shape
    rc = _load().oracle_fill_holes(img.ctypes.data, out.ctypes.data, h, w, int(conn))
    if rc != 0:
        raise ValueError("oracle_fill_holes failed with %d" % rc)
    return out


def recon_dilate_many(markers, masks, conn: int = 8) -> np.ndarray:
    """Reconstruction of a stack (n, h, w) of same-shaped images."""
    markers, masks = _u8(markers), _u8(masks)
    if markers.shape != masks.shape or markers.ndim != 3:
        raise ValueError("expected two (n, h, w) stacks of one shape")
    out = np.empty_like(markers)
    n, h, w = markers.shape
    rc = _load().oracle_recon_dilate_many(markers.ctypes.data, masks.ctypes.data,
                                          out.ctypes.data, n, h, w, int(conn))
    if rc != 0:
        raise ValueError("oracle_recon_dilate_many failed with %d" % rc)
    return out


def recon_erode(marker, mask, conn: int = 8) -> np.ndarray:
    """rho^e_mask(marker): reconstruction by erosion (marker raised over mask)."""
    marker, mask = _u8(marker), _u8(mask)
    if marker.shape != mask.shape or marker.ndim != 2:
        raise ValueError("marker and mask must be 2-D arrays of one shape")
    out = np.empty_like(marker)
    h, w = marker.shape
    rc = _load().oracle_recon_erode(marker.ctypes.data, mask.ctypes.data, out.ctypes.data, h, w, int(conn))
    if rc != 0:
        raise ValueError("oracle_recon_erode failed with %d" % rc)
    return out


def hdome(img, h: int, conn: int = 8) -> np.ndarray:
    """h-dome I - rho_I(max(I - h, 0)), h in 1..255."""
    img = _u8(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    out = np.empty_like(img)
    rc = _load().oracle_hdome(img.ctypes.data, out.ctypes.data, img.shape[0], img.shape[1], int(h), int(conn))
    if rc != 0:
        raise ValueError("oracle_hdome failed with %d" % rc)
    return out


def regional_max(img, conn: int = 8) -> np.ndarray:
    """Regional maxima: 255 where the 1-dome is positive, else 0."""
    img = _u8(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    out = np.empty_like(img)
    rc = _load().oracle_regional_max(img.ctypes.data, out.ctypes.data, img.shape[0], img.shape[1], int(conn))
    if rc != 0:
        raise ValueError("oracle_regional_max failed with %d" % rc)
    return out


def label(img, conn: int = 8):
    """Connected components of the nonzero pixels: (int32 labels 1..n in raster
    order of first pixels, 0 on the background; n)."""
    img = _u8(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    out = np.empty(img.shape, np.int32)
    n = _load().oracle_label(img.ctypes.data, out.ctypes.data, img.shape[0], img.shape[1], int(conn))
    if n < 0:
        raise ValueError("oracle_label failed")
    return out, int(n)


def area_threshold(img, min_area: int, max_area: int, conn: int = 8) -> np.ndarray:
    """255 on the components of the nonzero pixels whose area is in [min_area, max_area], else 0."""
    img = _u8(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    out = np.empty_like(img)
    n = _load().oracle_area_threshold(img.ctypes.data, out.ctypes.data, img.shape[0], img.shape[1], int(conn),
                                      int(min_area), int(max_area))
    if n < 0:
        raise ValueError("oracle_area_threshold failed")
    return out


def distance2(img) -> np.ndarray:
    """Squared Euclidean distance (int32) of every pixel to the nearest 0 pixel
    (2^31 - 1 if there is none)."""
    img = _u8(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    out = np.empty(img.shape, np.int32)
    if _load().oracle_distance2(img.ctypes.data, out.ctypes.data, img.shape[0], img.shape[1]) != 0:
        raise ValueError("oracle_distance2 failed")
    return out


def distance8(img) -> np.ndarray:
    """min(floor(sqrt(distance2)), 255) as uint8."""
    img = _u8(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    out = np.empty_like(img)
    if _load().oracle_distance8(img.ctypes.data, out.ctypes.data, img.shape[0], img.shape[1]) != 0:
        raise ValueError("oracle_distance8 failed")
    return out


def pre_watershed(img, conn: int = 8) -> np.ndarray:
    """Pre-Watershed markers: 255 on the regional maxima of distance8(img), else 0."""
    img = _u8(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    out = np.empty_like(img)
    if _load().oracle_pre_watershed(img.ctypes.data, out.ctypes.data, img.shape[0], img.shape[1], int(conn)) != 0:
        raise ValueError("oracle_pre_watershed failed")
    return out


def run_task(task) -> np.ndarray:
    """Oracle result of one task dict {op, marker/img, mask, conn} (host arrays)."""
    if task["op"] == "dilate":
        return recon_dilate(task["marker"], task["mask"], task["conn"])
    if task["op"] == "fill_holes":
        return fill_holes(task["img"], task["conn"])
    if task["op"] == "erode":
        return recon_erode(task["marker"], task["mask"], task["conn"])
    if task["op"] == "hdome":
        return hdome(task["img"], task["h"], task["conn"])
    if task["op"] == "regional_max":
        return regional_max(task["img"], task["conn"])
    raise ValueError("unknown op %r" % (task["op"],))
