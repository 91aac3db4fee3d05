"""Independent checks for the oracle, written straight from the mathematics.

Nothing here imports the oracle or the GPU library.

* ``iterate_definition``: the defining iteration of reconstruction by dilation,
  J_{n+1} = min(delta_B(J_n), I) from J_0 = min(J, I) until nothing changes,
  with delta_B the flat dilation by the 3x3 square (8-connectivity) or the
  cross (4-connectivity) and out-of-image pixels absent.  Vectorised over a
  leading batch axis so exhaustive sweeps of tiny images are cheap.
* ``threshold_decomposition``: the same result level by level through a
  library connected-component labelling (scipy.ndimage.label):
  rho(p) = max{h : p lies in a component of {I >= h} holding a pixel of
  {min(J, I) >= h}}.
* ``fill_holes_by_levels``: fill-holes through scipy's binary_fill_holes at
  every grey level t (its structure is the background connectivity):
  F(p) = max{t : p in fill({X >= t})}.
* ``iterate_erosion``: the defining iteration of reconstruction by erosion,
  J_{n+1} = max(eps_B(J_n), I) from max(J, I) (out-of-image pixels absent).
* ``regional_max_by_plateaus``: regional maxima straight from their
  definition, plateau by plateau through scipy.ndimage.label.
* ``label_by_propagation``: connected components of the nonzero pixels by
  propagating the smallest pixel index over foreground neighbours until
  nothing changes (the component's minimum index is its raster-first pixel),
  then numbering the components by that index.
"""
from __future__ import annotations

import numpy as np
import scipy.ndimage as ndi


def dilate(j: np.ndarray, conn: int) -> np.ndarray:
    """Flat dilation over the last two axes; pixels outside the image are absent."""
    j = np.asarray(j)
    pad = [(0, 0)] * (j.ndim - 2) + [(1, 1), (1, 1)]
    p = np.pad(j, pad, mode="constant", constant_values=0)
    h, w = j.shape[-2:]
    out = j.copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if conn == 4 and dy != 0 and dx != 0:
                continue
            out = np.maximum(out, p[..., 1 + dy:1 + dy + h, 1 + dx:1 + dx + w])
    return out


def iterate_definition(marker, mask, conn: int, max_iter: int | None = None):
    """Iterated elementary geodesic dilation to stability (batched over leading axes)."""
    mask = np.asarray(mask)
    j = np.minimum(np.asarray(marker), mask)
    n = 0
    while True:
        nxt = np.minimum(dilate(j, conn), mask)
        n += 1
        if np.array_equal(nxt, j):
            return j
        j = nxt
        if max_iter is not None and n >= max_iter:
            raise RuntimeError("no fixed point within max_iter")


def erode(j: np.ndarray, conn: int) -> np.ndarray:
    """Flat erosion over the last two axes; pixels outside the image are absent."""
    j = np.asarray(j)
    pad = [(0, 0)] * (j.ndim - 2) + [(1, 1), (1, 1)]
    p = np.pad(j, pad, mode="constant", constant_values=255)
    h, w = j.shape[-2:]
    out = j.copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if conn == 4 and dy != 0 and dx != 0:
                continue
            out = np.minimum(out, p[..., 1 + dy:1 + dy + h, 1 + dx:1 + dx + w])
    return out


def iterate_erosion(marker, mask, conn: int):
    """Iterated elementary geodesic erosion to stability: J <- max(erode(J), I) from max(J, I)."""
    mask = np.asarray(mask)
    j = np.maximum(np.asarray(marker), mask)
    while True:
        nxt = np.maximum(erode(j, conn), mask)
        if np.array_equal(nxt, j):
            return j
        j = nxt


def regional_max_by_plateaus(img, conn: int) -> np.ndarray:
    """Regional maxima from their definition: a connected plateau (one value,
    connectivity conn) none of whose neighbouring pixels is higher; 255 there.
    Plateaus at value 0 are left out (the reading the oracle states)."""
    img = np.asarray(img)
    out = np.zeros(img.shape, np.uint8)
    st = structure(conn)
    for v in np.unique(img):
        if v == 0:
            continue
        lab, n = ndi.label(img == v, structure=st)
        for k in range(1, n + 1):
            comp = lab == k
            ring = ndi.binary_dilation(comp, structure=st) & ~comp
            if not (img[ring] > v).any():
                out[comp] = 255
    return out


def structure(conn: int) -> np.ndarray:
    return ndi.generate_binary_structure(2, 1 if conn == 4 else 2)


def threshold_decomposition(marker, mask, conn: int) -> np.ndarray:
    """Reconstruction by labelling each upper level set of the mask."""
    mask = np.asarray(mask)
    j0 = np.minimum(np.asarray(marker), mask)
    out = np.zeros(mask.shape, dtype=np.uint8)
    st = structure(conn)
    for h in range(1, int(mask.max()) + 1 if mask.size else 1):
        lab, n = ndi.label(mask >= h, structure=st)
        if n == 0:
            break
        hit = np.unique(lab[(j0 >= h) & (lab > 0)])
        if hit.size == 0:
            continue
        keep = np.zeros(n + 1, dtype=bool)
        keep[hit] = True
        out[keep[lab]] = h
    return out


def fill_holes_binary(x, conn: int) -> np.ndarray:
    """255 * binary_fill_holes(x > 0) with the background connectivity ``conn``."""
    return np.where(ndi.binary_fill_holes(np.asarray(x) > 0, structure=structure(conn)),
                    255, 0).astype(np.uint8)


def fill_holes_by_levels(x, conn: int) -> np.ndarray:
    """Grey-level fill-holes as the stack of binary fills of each upper level set."""
    x = np.asarray(x)
    out = np.zeros(x.shape, dtype=np.uint8)
    st = structure(conn)
    for t in range(1, 256):
        filled = ndi.binary_fill_holes(x >= t, structure=st)
        if not filled.any():
            break
        out[filled] = t
    return out


def row_closed_form(marker_row, mask_row) -> np.ndarray:
    """One-row reconstruction: max of a left-to-right and a right-to-left pass."""
    i = np.asarray(mask_row).astype(np.int32)
    j = np.minimum(np.asarray(marker_row).astype(np.int32), i)
    n = len(i)
    fwd = np.zeros(n, np.int32)
    bwd = np.zeros(n, np.int32)
    acc = 0
    for x in range(n):
        acc = min(int(i[x]), max(int(j[x]), acc))
        fwd[x] = acc
    acc = 0
    for x in range(n - 1, -1, -1):
        acc = min(int(i[x]), max(int(j[x]), acc))
        bwd[x] = acc
    return np.maximum(fwd, bwd).astype(np.uint8)


def label_by_propagation(img, conn: int):
    """(labels, n) of the nonzero pixels of a 2-D image: each foreground pixel
    starts with its raster index and takes the minimum over its foreground
    neighbours (out-of-image pixels absent) until stable; components are then
    numbered 1..n in increasing order of that minimum."""
    fg = np.asarray(img) != 0
    h, w = fg.shape
    big = h * w
    cur = np.where(fg, np.arange(big, dtype=np.int64).reshape(h, w), big)
    while True:
        p = np.pad(cur, 1, mode="constant", constant_values=big)
        nxt = cur.copy()
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if conn == 4 and dy != 0 and dx != 0:
                    continue
                nxt = np.minimum(nxt, p[1 + dy:1 + dy + h, 1 + dx:1 + dx + w])
        nxt = np.where(fg, nxt, big)
        if np.array_equal(nxt, cur):
            break
        cur = nxt
    roots = np.unique(cur[fg])
    labels = np.zeros((h, w), np.int32)
    labels[fg] = np.searchsorted(roots, cur[fg]) + 1
    return labels, len(roots)
