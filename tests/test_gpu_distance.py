"""GPU parity of the exact distance transform and the Pre-Watershed markers
through the C ABI, against the CPU oracle (integer work: tolerance 0).

Inputs are seeded and synthetic: the binary nuclei tile (255 * (I > 120)),
random images of several densities, and the degenerate cases (no 0 pixel,
only 0 pixels, one 0 pixel far from most pixels, which caps D8 at 255).
"""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
CAP = 2 ** 31 - 1


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def lib(torch_mod):
    import paper_1209_3332_amd as p
    return p


@pytest.fixture(scope="module")
def rc(lib):
    ctx = lib.Recon(0)
    yield ctx
    ctx.close()


def dev(torch_mod, a):
    return torch_mod.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_distance(torch_mod, ctx, img):
    x = dev(torch_mod, img)
    d = ctx.distance(x)
    torch_mod.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), img), "the image must not be written"
    return d.cpu().numpy()


def gpu_markers(torch_mod, ctx, img, conn):
    x = dev(torch_mod, img)
    ctx.pre_watershed(x, conn)
    ctx.last_stats()
    return x.cpu().numpy()


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("%s: %d pixels differ, first at (%d, %d): got %d want %d"
                             % (what, len(bad), y, x, got[y, x], want[y, x]))


SHAPES = [(1, 1), (1, 300), (300, 1), (3, 257), (255, 256), (257, 255), (600, 90), (129, 1000)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_ragged_shapes(torch_mod, rc, oracle_mod, shape):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    for p in (0.5, 0.9, 0.99):
        img = np.where(rng.random(shape) < p, 255, 0).astype(np.uint8)
        assert_same(gpu_distance(torch_mod, rc, img), oracle_mod.distance2(img), "dist2 %s p %.2f" % (shape, p))
        for conn in (8, 4):
            assert_same(gpu_markers(torch_mod, rc, img, conn), oracle_mod.pre_watershed(img, conn),
                        "markers %s p %.2f conn %d" % (shape, p, conn))


@pytest.mark.parametrize("conn", [8, 4])
def test_nuclei_4096(torch_mod, rc, oracle_mod, conn):
    _, _, binary = synth.config2_tile()
    if conn == 8:
        assert_same(gpu_distance(torch_mod, rc, binary), oracle_mod.distance2(binary), "4096 nuclei dist2")
    m = gpu_markers(torch_mod, rc, binary, conn)
    assert_same(m, oracle_mod.pre_watershed(binary, conn), "4096 nuclei markers conn %d" % conn)
    assert (m > 0).sum() > 1000


def test_degenerate_images(torch_mod, rc, oracle_mod):
    for shape in [(1, 1), (7, 9), (300, 260)]:
        full = np.full(shape, 255, np.uint8)
        zero = np.zeros(shape, np.uint8)
        assert (gpu_distance(torch_mod, rc, full) == CAP).all()
        assert not gpu_distance(torch_mod, rc, zero).any()
        for conn in (8, 4):
            assert_same(gpu_markers(torch_mod, rc, full, conn), full, "no 0 pixel: one plateau at the cap")
            assert_same(gpu_markers(torch_mod, rc, zero, conn), zero, "only 0 pixels: no marker")
    # one 0 pixel: distances far beyond the D8 cap, long row searches
    one = np.full((1024, 1024), 255, np.uint8)
    one[700, 100] = 0
    assert_same(gpu_distance(torch_mod, rc, one), oracle_mod.distance2(one), "one 0 pixel")
    assert_same(gpu_markers(torch_mod, rc, one, 8), oracle_mod.pre_watershed(one, 8), "one 0 pixel markers")


def test_padded_views(torch_mod, rc, lib, oracle_mod):
    rng = np.random.default_rng(3)
    h, w = 301, 517
    img = np.where(rng.random((h, w)) < 0.93, 255, 0).astype(np.uint8)
    big = torch_mod.zeros((h + 2, w + 5), dtype=torch_mod.uint8, device="cuda")
    v = big[1:1 + h, 3:3 + w]
    v.copy_(torch_mod.from_numpy(img))
    plane = torch_mod.full((h, w + 9), -3, dtype=torch_mod.int32, device="cuda")
    d = plane[:, :w]
    rc.distance(v, d)
    torch_mod.cuda.synchronize()
    assert_same(d.cpu().numpy(), oracle_mod.distance2(img), "padded dist2")
    assert int((plane[:, w:] != -3).sum()) == 0
    rc.pre_watershed(v, 8)
    rc.last_stats()
    assert_same(v.cpu().numpy(), oracle_mod.pre_watershed(img, 8), "padded markers")
    assert int(big[0].sum()) == 0 and int(big[:, :3].sum()) == 0 and int(big[:, 3 + w:].sum()) == 0


def test_argument_errors(torch_mod, rc, lib):
    img = torch_mod.zeros((4, 5), dtype=torch_mod.uint8, device="cuda")
    d = torch_mod.zeros((4, 5), dtype=torch_mod.int32, device="cuda")
    with pytest.raises(lib.ReconError):
        rc.pre_watershed(img, 6)
    m = lib.image_of(img)
    L = lib.load_library()
    assert L.recon_distance(rc.ctx, ctypes.byref(m), d.data_ptr(), 4, None) == lib.RECON_EINVAL   # pitch < width
    wide = lib.recon_image(img.data_ptr(), 1, 20000, 20000)                                        # too wide
    assert L.recon_distance(rc.ctx, ctypes.byref(wide), d.data_ptr(), 20000, None) == lib.RECON_EINVAL
    assert L.recon_pre_watershed(rc.ctx, ctypes.byref(wide), 8, None) == lib.RECON_EINVAL
    alias = lib.recon_image(d.data_ptr(), 4, 5, 20)       # the image inside the distance plane
    assert L.recon_distance(rc.ctx, ctypes.byref(alias), d.data_ptr(), 5, None) == lib.RECON_EINVAL
    with pytest.raises(TypeError):
        rc.distance(img, torch_mod.zeros((4, 5), dtype=torch_mod.int64, device="cuda"))


def test_widest_rows(torch_mod, rc, oracle_mod):
    """Rows of the largest width (16384: a row of column distances fills 64 KiB of LDS)."""
    rng = np.random.default_rng(16384)
    img = np.where(rng.random((9, 16384)) < 0.995, 255, 0).astype(np.uint8)
    assert_same(gpu_distance(torch_mod, rc, img), oracle_mod.distance2(img), "16384-wide dist2")
    assert_same(gpu_markers(torch_mod, rc, img, 8), oracle_mod.pre_watershed(img, 8), "16384-wide markers")


def test_few_zero_pixels(torch_mod, rc):
    """Images with very few 0 pixels, where the distances are long and a
    search bounded only by each pixel's distance would cost O(width) per pixel:
    one 0 pixel in a corner of a 4096 x 4096 image, 0 pixels only along the
    first row, and a 16384-wide strip with a single 0 pixel.  Their distances
    have closed forms (the squared distance to the single 0 pixel, or to the
    first row), which the results must equal; the 4096 x 4096 one is timed too
    (it must stay a short kernel)."""
    import time
    corner = np.full((4096, 4096), 255, np.uint8)
    corner[0, 0] = 0
    yy, xx = np.indices(corner.shape, dtype=np.int64)
    assert_same(gpu_distance(torch_mod, rc, corner), (yy * yy + xx * xx).astype(np.int32), "corner dist2")
    top = np.full((1024, 2048), 255, np.uint8)
    top[0, :] = 0
    yy, _ = np.indices(top.shape, dtype=np.int64)
    assert_same(gpu_distance(torch_mod, rc, top), (yy * yy).astype(np.int32), "top-row dist2")
    strip = np.full((5, 16384), 255, np.uint8)
    strip[2, 9000] = 0
    yy, xx = np.indices(strip.shape, dtype=np.int64)
    assert_same(gpu_distance(torch_mod, rc, strip), ((yy - 2) ** 2 + (xx - 9000) ** 2).astype(np.int32),
                "strip dist2")
    x = torch_mod.from_numpy(corner).cuda()
    d = torch_mod.empty(corner.shape, dtype=torch_mod.int32, device="cuda")
    rc.distance(x, d)
    torch_mod.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        rc.distance(x, d)
    torch_mod.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    assert dt < 0.05, "one 0 pixel in 4096 x 4096 took %.3f s" % dt
