"""The HIP kernels' device code, compiled for the CPU and run on emulated waves,
must equal the oracle (no GPU needed).

tests/kernel_emu compiles paper_1209_3332_amd/csrc/kernels.hpp against a
stand-in HIP header: each 64-lane wave runs as fibers on its own OS thread,
so the block scheduler runs with real concurrency, and the build uses
AddressSanitizer + UBSan so that every LDS and global access of the kernels
is bounds-checked.  This is where kernel logic is debugged before it runs on
the GPU.
"""
import numpy as np
import pytest

import kemu
import synth


@pytest.fixture(scope="session")
def emu_exe(tmp_path_factory):
    return kemu.build(str(tmp_path_factory.mktemp("kemu")), sanitize=True)


def _check(exe, oracle_mod, tasks, **kw):
    rc, outs, log = kemu.run(exe, tasks, **kw)
    assert rc == 0, log[-2000:]
    assert "ERROR: AddressSanitizer" not in log and "runtime error" not in log, log[-2000:]
    for k, (t, got) in enumerate(zip(tasks, outs)):
        want = oracle_mod.run_task(t)
        assert got is not None and np.array_equal(got, want), "task %d (%s, conn %d) differs in %d px" % (
            k, t["op"], t["conn"], -1 if got is None else int((got != want).sum()))
    return log


@pytest.mark.parametrize("conn", [8, 4])
def test_small_shapes(emu_exe, oracle_mod, conn):
    rng = np.random.default_rng(10 + conn)
    tasks = []
    for (h, w) in [(1, 1), (1, 9), (9, 1), (2, 3), (7, 300), (33, 257)]:
        m, k = synth.random_pair(rng, h, w, 3)   # unclipped markers (marker > mask in places)
        tasks.append({"op": "dilate", "marker": m, "mask": k, "conn": conn})
    _check(emu_exe, oracle_mod, tasks, n_waves=3)


@pytest.mark.parametrize("conn", [8, 4])
def test_nuclei_crop(emu_exe, oracle_mod, conn):
    marker, mask, _ = synth.config2_tile(seed=synth.seed_for(2, 21), size=96, n_gauss=2)
    mask = np.ascontiguousarray(np.concatenate([mask, mask[:, ::-1]], 1))[:, :300]
    marker = synth.hdome_marker(mask, 20)
    _check(emu_exe, oracle_mod, [{"op": "dilate", "marker": marker, "mask": mask, "conn": conn}], n_waves=4)


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_holes(emu_exe, oracle_mod, conn):
    rng = np.random.default_rng(40 + conn)
    tasks = [{"op": "fill_holes", "img": np.where(rng.random((40, 300)) < 0.6, 255, 0).astype(np.uint8),
              "conn": conn},
             {"op": "fill_holes", "img": rng.integers(0, 256, (20, 270)).astype(np.uint8), "conn": conn},
             {"op": "fill_holes", "img": np.array([[0, 0, 0], [0, 9, 0], [0, 0, 0]], np.uint8), "conn": conn}]
    _check(emu_exe, oracle_mod, tasks, n_waves=3)


@pytest.mark.parametrize("conn", [8, 4])
def test_erode_hdome_regional_max(emu_exe, oracle_mod, conn):
    """Reconstruction by erosion, h-dome and regional maxima: ragged shapes,
    a grey nuclei crop, unclipped markers and plateaus."""
    rng = np.random.default_rng(60 + conn)
    _, grey, _ = synth.config2_tile(seed=synth.seed_for(2, 24), size=96, n_gauss=2)
    grey = np.ascontiguousarray(np.concatenate([grey, grey[:, ::-1]], 1))[:, :270]
    tasks = []
    for (h, w) in [(1, 1), (9, 1), (33, 257)]:
        m, k = synth.random_pair(rng, h, w, 5)
        tasks.append({"op": "erode", "marker": m, "mask": k, "conn": conn})
    tasks.append({"op": "erode", "marker": np.full_like(grey, 255), "mask": grey, "conn": conn})
    tasks.append({"op": "hdome", "img": grey, "h": 30, "conn": conn})
    tasks.append({"op": "hdome", "img": rng.integers(0, 256, (20, 270)).astype(np.uint8), "h": 255,
                  "conn": conn})
    tasks.append({"op": "regional_max", "img": grey, "conn": conn})
    tasks.append({"op": "regional_max", "img": rng.integers(0, 4, (40, 300)).astype(np.uint8), "conn": conn})
    tasks.append({"op": "regional_max", "img": np.zeros((5, 7), np.uint8), "conn": conn})
    _check(emu_exe, oracle_mod, tasks, n_waves=3)


def test_staged_pipeline(emu_exe, oracle_mod):
    """The staged pipeline (dense pass, border seeding and revisits as separate
    kernels) run to the end gives the same bytes as the persistent one."""
    marker, mask, binary = synth.config2_tile(seed=synth.seed_for(2, 23), size=96, n_gauss=2)
    mask = np.ascontiguousarray(np.concatenate([mask, mask[:, ::-1]], 1))[:, :300]
    marker = synth.hdome_marker(mask, 20)
    img = np.where(mask > 40, 255, 0).astype(np.uint8)
    tasks = [{"op": "dilate", "marker": marker, "mask": mask, "conn": 8},
             {"op": "fill_holes", "img": img, "conn": 4},
             {"op": "erode", "marker": np.full_like(mask, 255), "mask": mask, "conn": 4},
             {"op": "hdome", "img": mask, "h": 20, "conn": 8}]
    _check(emu_exe, oracle_mod, tasks, n_waves=3, stop_after=3)


def test_large_batch_table_in_memory(emu_exe, oracle_mod):
    # more tasks than fit in the kernel arguments: the table lives in memory
    rng = np.random.default_rng(77)
    tasks = []
    for i in range(14):
        h, w = int(rng.integers(1, 40)), int(rng.integers(1, 300))
        conn = int(rng.choice([4, 8]))
        if i % 4 == 3:
            tasks.append({"op": "fill_holes", "img": np.where(rng.random((h, w)) < 0.6, 255, 0).astype(np.uint8),
                          "conn": conn})
        else:
            m, k = synth.random_pair(rng, h, w, 4)
            tasks.append({"op": "dilate", "marker": m, "mask": k, "conn": conn})
    _check(emu_exe, oracle_mod, tasks, n_waves=4)


@pytest.mark.parametrize("bh,qcap", [(16, 2048), (64, 2048), (32, 64)])
def test_block_shapes_and_queue_overflow(emu_exe, oracle_mod, bh, qcap):
    rng = np.random.default_rng(bh + qcap)
    mask = rng.integers(0, 256, (70, 270)).astype(np.uint8)
    tasks = [{"op": "dilate", "marker": synth.hdome_marker(mask, 40), "mask": mask, "conn": 8},
             {"op": "dilate", "marker": synth.hdome_marker(mask, 40), "mask": mask, "conn": 4}]
    log = _check(emu_exe, oracle_mod, tasks, bh=bh, qcap=qcap, scan_rounds=0, n_waves=3)
    if qcap == 64:
        assert "overflow 0 " not in log   # the overflow path was exercised


def test_spiral_chain(emu_exe, oracle_mod):
    marker, mask, _ = synth.spiral_tile(40, 520, "inner")
    _check(emu_exe, oracle_mod, [{"op": "dilate", "marker": marker, "mask": mask, "conn": 8},
                                 {"op": "dilate", "marker": marker, "mask": mask, "conn": 4}], n_waves=3)


def test_dense_pass_is_blockwise_reconstruction(emu_exe, oracle_mod):
    # after K1 alone, each 32 x 256 block holds its own reconstruction (empty halo)
    rng = np.random.default_rng(5)
    mask = rng.integers(0, 256, (70, 600)).astype(np.uint8)
    marker = synth.hdome_marker(mask, 50)
    rc, outs, log = kemu.run(emu_exe, [{"op": "dilate", "marker": marker, "mask": mask, "conn": 8}],
                             n_waves=2, stop_after=1)
    assert rc == 0, log[-2000:]
    want = np.empty_like(mask)
    for y0 in range(0, 70, 32):
        for x0 in range(0, 600, 256):
            sl = np.s_[y0:y0 + 32, x0:x0 + 256]
            want[sl] = oracle_mod.recon_dilate(marker[sl], mask[sl], 8)
    assert np.array_equal(outs[0], want)


@pytest.mark.parametrize("conn", [8, 4])
def test_label_and_area_threshold(emu_exe, oracle_mod, conn):
    """Connected-component labelling (tile-local union-find, merges across
    tiles, rank relabelling) and the area filter, against the oracle: ragged
    shapes spanning several 16 x 256 tiles, densities around the percolation
    threshold, checkerboards, a spiral corridor crossing tiles, a nuclei crop."""
    rng = np.random.default_rng(90 + conn)
    imgs = [np.zeros((1, 1), np.uint8), np.full((3, 5), 7, np.uint8)]
    for (h, w, p) in [(17, 300, 0.5), (40, 520, 0.62), (70, 260, 0.45), (33, 257, 0.9)]:
        imgs.append(np.where(rng.random((h, w)) < p, 255, 0).astype(np.uint8))
    yy, xx = np.mgrid[0:35, 0:300]
    imgs.append(np.where((yy + xx) % 2 == 0, 255, 0).astype(np.uint8))
    # thin diagonal lines crossing tile rows and columns anywhere, corners included
    yy, xx = np.mgrid[0:50, 0:600]
    imgs.append(np.where((xx - yy) % 7 == 0, 255, 0).astype(np.uint8))
    imgs.append(np.where(((xx + yy) % 5 == 0) | ((xx - 2 * yy) % 13 == 0), 255, 0).astype(np.uint8))
    imgs.append(synth.spiral_tile(40, 520, "outer")[1])
    _, _, binary = synth.config2_tile(seed=synth.seed_for(2, 25), size=96, n_gauss=2)
    imgs.append(np.ascontiguousarray(np.concatenate([binary, binary[:, ::-1], binary], 1)))
    for i, img in enumerate(imgs):
        rc, lab, count, area, log = kemu.run_label(emu_exe, img, conn, min_area=3, max_area=40, n_waves=3)
        assert rc == 0, log[-2000:]
        assert "ERROR: AddressSanitizer" not in log and "runtime error" not in log, log[-2000:]
        want, n = oracle_mod.label(img, conn)
        assert count == n, (i, count, n)
        assert np.array_equal(lab, want), "image %d: %d labels differ" % (i, int((lab != want).sum()))
        assert np.array_equal(area, oracle_mod.area_threshold(img, 3, 40, conn)), "image %d area filter" % i


def test_distance_transform(emu_exe, oracle_mod):
    """Column segments (with carries from outside the segment) and the row
    search, against the oracle's exact squared distances and capped D8."""
    rng = np.random.default_rng(77)
    imgs = [np.zeros((1, 1), np.uint8), np.full((1, 1), 5, np.uint8), np.full((3, 7), 9, np.uint8)]
    for (h, w, p) in [(300, 40, 0.9), (530, 23, 0.995), (17, 300, 0.7), (260, 270, 0.97)]:
        imgs.append(np.where(rng.random((h, w)) < p, 255, 0).astype(np.uint8))
    one = np.full((600, 5), 255, np.uint8)
    one[599, 2] = 0                     # distances beyond 255: the D8 cap, carries across segments
    imgs.append(one)
    # rows of several anchor segments (a last pixel that is, or is not, an anchor itself)
    # with few 0 pixels, where the anchors' columns bound every other pixel's search
    for (h, w, zeros) in [(3, 257, [(0, 256)]), (2, 513, [(1, 0)]), (5, 1030, [(4, 1029)]),
                          (4, 1100, [(0, 0), (3, 700)]), (3, 769, [])]:
        im = np.full((h, w), 255, np.uint8)
        for zy, zx in zeros:
            im[zy, zx] = 0
        imgs.append(im)
    top = np.full((40, 600), 255, np.uint8)
    top[0, :] = 0                       # 0 pixels only in the first row: g = y everywhere
    imgs.append(top)
    imgs.append(np.where(rng.random((6, 1300)) < 0.999, 255, 0).astype(np.uint8))
    _, _, binary = synth.config2_tile(seed=synth.seed_for(2, 26), size=96, n_gauss=2)
    imgs.append(binary)
    for i, img in enumerate(imgs):
        rc, d2, d8, log = kemu.run_edt(emu_exe, img)
        assert rc == 0, log[-2000:]
        assert "ERROR: AddressSanitizer" not in log and "runtime error" not in log, log[-2000:]
        assert np.array_equal(d2, oracle_mod.distance2(img)), "image %d dist2" % i
        assert np.array_equal(d8, oracle_mod.distance8(img)), "image %d D8" % i


def test_failed_claims_abort_the_launch(emu_exe):
    """A block claim whose compare-and-swap keeps failing gives the launch up
    (abort flag set, every wave leaves) instead of working on a block the wave
    does not own.  The test hook makes every claim fail from the host."""
    rng = np.random.default_rng(77)
    m, k = synth.random_pair(rng, 70, 300, 4)
    rc, _, log = kemu.run(emu_exe, [{"op": "dilate", "marker": m, "mask": k, "conn": 8}], n_waves=3,
                          test_fault=1, timeout=120)
    assert "ERROR: AddressSanitizer" not in log and "runtime error" not in log, log[-2000:]
    assert rc != 0 and "rc -3" in log and "aborted 1" in log, log[-2000:]


def _route_count(log):
    return int(log.split(" route ")[1].split()[0])


@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("bh", [16, 32, 64])
def test_component_route(emu_exe, oracle_mod, conn, bh):
    """Two-valued masks take the component route (labelling and a maximum per
    component), grey ones the block route, in one launch; every result equals
    the oracle.  Covers binary dilation with grey markers, markers above the
    mask, a mask of one nonzero value other than 255, all-zero and constant
    masks, fill-holes (complemented mask), erosion, h-dome and regional maxima
    of binary images, spirals, ragged shapes and tiles wider than one block."""
    rng = np.random.default_rng(900 + conn + bh)
    tasks = []
    two_valued = 0
    for (h, w) in [(1, 1), (1, 9), (9, 1), (37, 300), (70, 530)]:
        mask = np.where(rng.random((h, w)) < 0.55, 255, 0).astype(np.uint8)
        marker = rng.integers(0, 256, (h, w)).astype(np.uint8) * (rng.random((h, w)) < 0.02)
        tasks.append({"op": "dilate", "marker": marker, "mask": mask, "conn": conn})
        two_valued += 1
    m7 = np.where(rng.random((50, 260)) < 0.6, 7, 0).astype(np.uint8)          # {0, 7}, markers above it
    tasks.append({"op": "dilate", "marker": rng.integers(0, 256, (50, 260)).astype(np.uint8), "mask": m7,
                  "conn": conn})
    tasks.append({"op": "dilate", "marker": rng.integers(0, 9, (20, 40)).astype(np.uint8),
                  "mask": np.zeros((20, 40), np.uint8), "conn": conn})                # all zero
    tasks.append({"op": "dilate", "marker": (rng.random((30, 270)) < 0.001).astype(np.uint8) * 9,
                  "mask": np.full((30, 270), 200, np.uint8), "conn": conn})           # constant
    two_valued += 3
    spiral, seed = synth.spiral_tile(61, 300, "inner")[:2]
    tasks.append({"op": "dilate", "marker": seed, "mask": spiral, "conn": conn})
    two_valued += 1
    binary = np.where(rng.random((66, 300)) < 0.6, 255, 0).astype(np.uint8)
    tasks.append({"op": "fill_holes", "img": binary, "conn": conn})
    tasks.append({"op": "erode", "marker": np.full_like(binary, 255), "mask": binary, "conn": conn})
    tasks.append({"op": "hdome", "img": binary, "h": 40, "conn": conn})
    tasks.append({"op": "regional_max", "img": binary, "conn": conn})
    two_valued += 4
    m, k = synth.random_pair(rng, 40, 300, 5)                   # grey: the block route
    tasks.append({"op": "dilate", "marker": m, "mask": k, "conn": conn})
    tasks.append({"op": "fill_holes", "img": rng.integers(0, 256, (20, 270)).astype(np.uint8), "conn": conn})
    log = _check(emu_exe, oracle_mod, tasks, n_waves=3, bh=bh, component=1)
    assert _route_count(log) == two_valued, log[-500:]


def test_component_route_policy(emu_exe, oracle_mod):
    """The default policy: beside a grey task, a thick two-valued mask (the
    fill-holes of blobs) keeps the block route and a thin one (a corridor)
    takes the component route; alone, the thick one takes the route too.
    Every result equals the oracle either way."""
    rng = np.random.default_rng(5150)
    m, k = synth.random_pair(rng, 40, 300, 5)
    grey = {"op": "dilate", "marker": m, "mask": k, "conn": 8}
    yy, xx = np.mgrid[0:64, 0:300]
    blobs = np.where(((yy % 32) - 16) ** 2 + ((xx % 40) - 20) ** 2 < 60, 255, 0).astype(np.uint8)
    thick = {"op": "fill_holes", "img": blobs, "conn": 8}
    spiral, seed = synth.spiral_tile(61, 300, "outer")[:2]
    thin = {"op": "dilate", "marker": seed, "mask": spiral, "conn": 4}
    log = _check(emu_exe, oracle_mod, [grey, thick, thin], n_waves=3, component=2)
    assert _route_count(log) == 1, log[-500:]
    log = _check(emu_exe, oracle_mod, [thick], n_waves=3, component=2)
    assert _route_count(log) == 1, log[-500:]
    log = _check(emu_exe, oracle_mod, [grey, thick], n_waves=3, component=2)
    assert _route_count(log) == 0, log[-500:]
    # a mask whose sample looks two-valued but that is grey off the sampled
    # pixels: the classification reads it whole and keeps it on the block
    # route, and (grey work after all) the thick mask beside it too, unless
    # the policy sends every two-valued mask to the route
    sneaky_mask = np.full((64, 300), 255, np.uint8)
    sneaky_mask[0, :5] = 100
    sneaky = {"op": "dilate", "marker": synth.hdome_marker(sneaky_mask, 30), "mask": sneaky_mask, "conn": 8}
    for mode, routed in ((2, 0), (1, 1)):
        log = _check(emu_exe, oracle_mod, [sneaky, thick], n_waves=3, component=mode)
        assert _route_count(log) == routed, (mode, log[-500:])


def _stat(log, name):
    return int(log.split(" %s " % name)[1].split()[0])


@pytest.mark.parametrize("spill", [8192, 64])
def test_spill_queue(emu_exe, oracle_mod, spill):
    """A 64-entry LDS queue with the global spill queue under it: with a large
    spill, pushes that do not fit the LDS ring go to the spill and come back
    through the drain, with no re-seed; with a 64-entry spill both fill up and
    the block re-seeds.  The bytes equal the oracle's either way."""
    rng = np.random.default_rng(7000 + spill)
    mask = rng.integers(0, 256, (70, 270)).astype(np.uint8)
    tasks = [{"op": "dilate", "marker": synth.hdome_marker(mask, 40), "mask": mask, "conn": 8},
             {"op": "dilate", "marker": synth.hdome_marker(mask, 40), "mask": mask, "conn": 4},
             {"op": "fill_holes", "img": np.where(rng.random((60, 300)) < 0.6, 255, 0).astype(np.uint8),
              "conn": 4}]
    log = _check(emu_exe, oracle_mod, tasks, qcap=64, scan_rounds=0, n_waves=3, spill=spill)
    assert _stat(log, "spill") > 0, log[-300:]
    if spill == 8192:
        assert _stat(log, "overflow") == 0, log[-300:]
    else:
        assert _stat(log, "overflow") > 0, log[-300:]
