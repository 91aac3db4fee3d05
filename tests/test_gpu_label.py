"""GPU parity of connected-component labelling (BWLabel) and the area filter
(AreaThreshold) through the C ABI, against the CPU oracle.

Labels are numbered in raster order of each component's first pixel on both
sides, so the comparison is element by element (integer work: tolerance 0),
and so is the component count.  Inputs are seeded and synthetic: the binary
nuclei tile (255 * (I > 120)) of the reconstruction workloads, random images
around the percolation threshold, checkerboards (the most components), a
full image (one component of every pixel) and the spiral corridor (one
component threading every tile).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


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


def gpu_label(torch_mod, ctx, img, conn):
    x = dev(torch_mod, img)
    count = torch_mod.full((1,), -1, dtype=torch_mod.int32, device="cuda")
    lab = ctx.label(x, conn=conn, count=count)
    torch_mod.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), img), "the image must not be written"
    return lab.cpu().numpy(), int(count.item())


def gpu_area(torch_mod, ctx, img, lo, hi, conn):
    x = dev(torch_mod, img)
    ctx.area_threshold(x, lo, hi, conn)
    torch_mod.cuda.synchronize()
    return x.cpu().numpy()


def check_label(torch_mod, ctx, oracle_mod, img, conn, what):
    got, n = gpu_label(torch_mod, ctx, img, conn)
    want, wn = oracle_mod.label(img, conn)
    assert n == wn, "%s: %d components, oracle %d" % (what, n, wn)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("%s: %d labels differ, first at (%d, %d): got %d want %d"
                             % (what, len(bad), y, x, got[y, x], want[y, x]))
    return n


SHAPES = [(1, 1), (1, 300), (300, 1), (2, 2), (15, 255), (16, 256), (17, 257), (33, 520), (100, 513), (257, 131)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
@pytest.mark.parametrize("conn", [8, 4])
def test_ragged_shapes(torch_mod, rc, oracle_mod, shape, conn):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1] + conn)
    for p in (0.3, 0.5, 0.6, 0.95):
        img = np.where(rng.random(shape) < p, 255, 0).astype(np.uint8)
        check_label(torch_mod, rc, oracle_mod, img, conn, "%s p %.2f conn %d" % (shape, p, conn))
        lo, hi = sorted(int(v) for v in rng.integers(1, 30, 2))
        assert np.array_equal(gpu_area(torch_mod, rc, img, lo, hi, conn),
                              oracle_mod.area_threshold(img, lo, hi, conn)), "area %s [%d, %d]" % (shape, lo, hi)


@pytest.mark.parametrize("conn", [8, 4])
def test_nuclei_4096(torch_mod, rc, oracle_mod, conn):
    _, _, binary = synth.config2_tile()
    n = check_label(torch_mod, rc, oracle_mod, binary, conn, "4096 nuclei conn %d" % conn)
    assert n > 1000
    assert np.array_equal(gpu_area(torch_mod, rc, binary, 20, 1000, conn),
                          oracle_mod.area_threshold(binary, 20, 1000, conn)), "4096 nuclei area filter"


@pytest.mark.parametrize("conn", [8, 4])
def test_adversarial_4096(torch_mod, rc, oracle_mod, conn):
    rng = np.random.default_rng(4096 + conn)
    # around the percolation threshold: components of every size, spanning many tiles
    noise = np.where(rng.random((4096, 4096)) < (0.59 if conn == 4 else 0.41), 255, 0).astype(np.uint8)
    check_label(torch_mod, rc, oracle_mod, noise, conn, "percolating noise conn %d" % conn)
    full = np.full((4096, 4096), 255, np.uint8)
    got, n = gpu_label(torch_mod, rc, full, conn)
    assert n == 1 and (got == 1).all()
    yy, xx = np.mgrid[0:4096, 0:4096]
    cb = np.where((yy + xx) % 2 == 0, 255, 0).astype(np.uint8)
    n = check_label(torch_mod, rc, oracle_mod, cb, conn, "checkerboard conn %d" % conn)
    assert n == (4096 * 4096 // 2 if conn == 4 else 1)
    _, corridor, _ = synth.spiral_tile(4096, 4096, "outer")
    got, n = gpu_label(torch_mod, rc, corridor, conn)
    assert n == 1 and np.array_equal(got > 0, corridor > 0) and got.max() == 1


def test_padded_views_and_pitch(torch_mod, rc, lib, oracle_mod):
    rng = np.random.default_rng(11)
    h, w = 70, 301
    img = np.where(rng.random((h, w)) < 0.55, 255, 0).astype(np.uint8)
    big = torch_mod.zeros((h + 1, w + 7), dtype=torch_mod.uint8, device="cuda")
    v = big[1:, 3:3 + w]
    v.copy_(torch_mod.from_numpy(img))
    plane = torch_mod.full((h, w + 13), -7, dtype=torch_mod.int32, device="cuda")
    lab = plane[:, :w]
    for conn in (4, 8):
        rc.label(v, lab, conn)
        torch_mod.cuda.synchronize()
        want, _ = oracle_mod.label(img, conn)
        assert np.array_equal(lab.cpu().numpy(), want)
        assert int((plane[:, w:] != -7).sum()) == 0, "the label plane's padding was written"
        x = big.clone()
        xv = x[1:, 3:3 + w]
        rc.area_threshold(xv, 2, 50, conn)
        torch_mod.cuda.synchronize()
        assert np.array_equal(xv.cpu().numpy(), oracle_mod.area_threshold(img, 2, 50, conn))
        assert int(x[0].sum()) == 0 and int(x[:, :3].sum()) == 0 and int(x[:, 3 + w:].sum()) == 0


def test_area_bounds(torch_mod, rc, oracle_mod):
    _, _, binary = synth.config2_tile(seed=synth.seed_for(2, 32), size=1024, n_gauss=188)
    for conn in (8, 4):
        for lo, hi in [(0, 0), (1, 1), (0, 1 << 40), (50, 50), (100, 400), (1 << 30, 1 << 40)]:
            assert np.array_equal(gpu_area(torch_mod, rc, binary, lo, hi, conn),
                                  oracle_mod.area_threshold(binary, lo, hi, conn)), (conn, lo, hi)


def test_determinism_and_reuse(torch_mod, rc, oracle_mod):
    rng = np.random.default_rng(12)
    img = np.where(rng.random((1500, 1700)) < 0.45, 255, 0).astype(np.uint8)
    first, n = gpu_label(torch_mod, rc, img, 8)
    for _ in range(3):
        again, n2 = gpu_label(torch_mod, rc, img, 8)
        assert n2 == n and np.array_equal(again, first)
    # a smaller image afterwards reuses the workspace
    small = img[:100, :90].copy()
    check_label(torch_mod, rc, oracle_mod, small, 8, "small after large")


def test_argument_errors(torch_mod, rc, lib):
    img = torch_mod.zeros((4, 5), dtype=torch_mod.uint8, device="cuda")
    lab = torch_mod.zeros((4, 5), dtype=torch_mod.int32, device="cuda")
    with pytest.raises(lib.ReconError):
        rc.label(img, lab, 6)
    with pytest.raises(lib.ReconError):
        rc.area_threshold(img, 5, 4)            # min above max
    with pytest.raises(lib.ReconError):
        rc.area_threshold(img, -1, 4)
    with pytest.raises(TypeError):
        rc.label(img, torch_mod.zeros((4, 6), dtype=torch_mod.int32, device="cuda"))
    import ctypes
    m = lib.image_of(img)
    assert lib.load_library().recon_label(rc.ctx, ctypes.byref(m), lab.data_ptr(), 3, 8, None, None) == lib.RECON_EINVAL
    alias = lib.recon_image(lab.data_ptr(), 4, 5, 20)     # the image inside the label plane
    assert lib.load_library().recon_label(rc.ctx, ctypes.byref(alias), lab.data_ptr(), 5, 8, None,
                                          None) == lib.RECON_EINVAL
    rc.label(img, lab, 8)                        # nothing was enqueued by the failures
    torch_mod.cuda.synchronize()
    assert int(lab.abs().sum()) == 0


def test_max_size_tile(torch_mod, rc, oracle_mod):
    """The largest tile of the tests: 16384 x 16384, the binary nuclei image of
    the generator scaled to its area (65536 tiles of 16 x 256)."""
    mask = synth.scaled_config1_tile(16384, 16384, synth.seed_for(6, 1))
    binary = np.where(mask > 60, 255, 0).astype(np.uint8)
    n = check_label(torch_mod, rc, oracle_mod, binary, 8, "16384 nuclei labels")
    assert n > 10000
    assert np.array_equal(gpu_area(torch_mod, rc, binary, 20, 1000, 8),
                          oracle_mod.area_threshold(binary, 20, 1000, 8)), "16384 area filter"
