"""GPU parity of the operations built on the same kernels: reconstruction by
erosion, h-dome and regional maxima, through the C ABI, against the CPU oracle
byte for byte (integer work: tolerance 0).

Inputs are seeded and synthetic: the nuclei tiles and ragged random pairs of
the dilation tests; erosion markers are the mask raised by h (the dual of the
h-dome marker), so that the erosion floods down from above.
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


def raised(mask, h):
    """Erosion marker: the mask raised by h, capped at 255."""
    return np.minimum(mask.astype(np.int32) + h, 255).astype(np.uint8)


def gpu_erode(torch_mod, ctx, marker, mask, conn):
    m, k = dev(torch_mod, marker), dev(torch_mod, mask)
    ctx.erode(m, k, conn)
    ctx.last_stats()   # waits with a deadline; raises if the launch was stopped
    return m.cpu().numpy()


def gpu_hdome(torch_mod, ctx, img, h, conn):
    x = dev(torch_mod, img)
    ctx.hdome(x, h, conn)
    ctx.last_stats()
    return x.cpu().numpy()


def gpu_rmax(torch_mod, ctx, img, conn):
    x = dev(torch_mod, img)
    ctx.regional_max(x, conn)
    ctx.last_stats()
    return x.cpu().numpy()


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("%s: %d pixels differ, first at (%d, %d): got %d want %d"
                             % (what, len(bad), y, x, got[y, x], want[y, x]))


SHAPES = [(1, 1), (1, 7), (7, 1), (1, 300), (300, 1), (3, 257), (33, 257), (64, 512), (257, 131), (129, 1000)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
@pytest.mark.parametrize("conn", [8, 4])
def test_erode_ragged_shapes(torch_mod, rc, oracle_mod, shape, conn):
    rng = np.random.default_rng(7000 + shape[0] * 1000 + shape[1] + conn)
    for levels in (3, 256):
        marker, mask = synth.random_pair(rng, shape[0], shape[1], levels)   # marker below mask in places
        if levels == 256:
            marker = raised(mask, int(rng.integers(1, 80)))
        assert_same(gpu_erode(torch_mod, rc, marker, mask, conn), oracle_mod.recon_erode(marker, mask, conn),
                    "erode %dx%d levels %d conn %d" % (shape[0], shape[1], levels, conn))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
@pytest.mark.parametrize("conn", [8, 4])
def test_hdome_and_regional_max_ragged(torch_mod, rc, oracle_mod, shape, conn):
    rng = np.random.default_rng(8000 + shape[0] * 1000 + shape[1] + conn)
    img = rng.integers(0, 256, size=shape).astype(np.uint8)
    h = int(rng.integers(1, 256))
    assert_same(gpu_hdome(torch_mod, rc, img, h, conn), oracle_mod.hdome(img, h, conn),
                "hdome %s h %d conn %d" % (shape, h, conn))
    few = rng.integers(0, 4, size=shape).astype(np.uint8)   # many plateaus
    assert_same(gpu_rmax(torch_mod, rc, few, conn), oracle_mod.regional_max(few, conn),
                "regional max %s conn %d" % (shape, conn))


@pytest.mark.parametrize("conn", [8, 4])
def test_nuclei_1024(torch_mod, rc, oracle_mod, conn):
    _, mask, _ = synth.config2_tile(seed=synth.seed_for(2, 8), size=1024, n_gauss=188)
    marker = raised(mask, 30)
    assert_same(gpu_erode(torch_mod, rc, marker, mask, conn), oracle_mod.recon_erode(marker, mask, conn),
                "1024 nuclei erode conn %d" % conn)
    for h in (1, 30, 255):
        assert_same(gpu_hdome(torch_mod, rc, mask, h, conn), oracle_mod.hdome(mask, h, conn),
                    "1024 nuclei hdome %d conn %d" % (h, conn))
    assert_same(gpu_rmax(torch_mod, rc, mask, conn), oracle_mod.regional_max(mask, conn),
                "1024 nuclei regional max conn %d" % conn)


@pytest.mark.parametrize("conn", [8, 4])
def test_full_4096_tile(torch_mod, rc, oracle_mod, conn):
    marker, mask, _ = synth.config2_tile()
    assert_same(gpu_hdome(torch_mod, rc, mask, 30, conn), oracle_mod.hdome(mask, 30, conn),
                "4096 nuclei hdome conn %d" % conn)
    # the tile's marker is max(I - 20, 0): its h-dome is I minus the dilation result
    assert_same(gpu_hdome(torch_mod, rc, mask, 20, conn), mask - oracle_mod.recon_dilate(marker, mask, conn),
                "4096 nuclei hdome vs dilation conn %d" % conn)
    up = raised(mask, 30)
    assert_same(gpu_erode(torch_mod, rc, up, mask, conn), oracle_mod.recon_erode(up, mask, conn),
                "4096 nuclei erode conn %d" % conn)
    assert_same(gpu_rmax(torch_mod, rc, mask, conn), oracle_mod.regional_max(mask, conn),
                "4096 nuclei regional max conn %d" % conn)


def test_degenerate_images(torch_mod, rc, oracle_mod):
    for conn in (8, 4):
        for shape in [(1, 1), (5, 7), (40, 300)]:
            zero = np.zeros(shape, np.uint8)
            flat = np.full(shape, 77, np.uint8)
            full = np.full(shape, 255, np.uint8)
            assert_same(gpu_rmax(torch_mod, rc, zero, conn), zero, "all-zero image has no maxima")
            assert_same(gpu_rmax(torch_mod, rc, flat, conn), full, "a flat image is one maximum")
            assert_same(gpu_hdome(torch_mod, rc, flat, 255, conn), flat, "255-dome of a flat image")
            assert_same(gpu_hdome(torch_mod, rc, flat, 1, conn), np.ones(shape, np.uint8), "1-dome, flat")
            # no low marker pixel: nothing erodes; one low pixel floods the flat mask
            assert_same(gpu_erode(torch_mod, rc, full, zero, conn), full, "erode 255 over 0")
            seed = full.copy()
            seed[shape[0] // 2, shape[1] // 2] = 0
            assert_same(gpu_erode(torch_mod, rc, seed, zero, conn), zero, "erode from one seed over 0")
            assert_same(gpu_erode(torch_mod, rc, zero, flat, conn), flat, "marker below mask -> mask")


def test_unaligned_views(torch_mod, rc, oracle_mod):
    rng = np.random.default_rng(44)
    h, w = 90, 301
    _, mask = synth.random_pair(rng, h, w, 256)
    marker = raised(mask, 25)
    big_m = torch_mod.zeros((h, w + 7), dtype=torch_mod.uint8, device="cuda")
    big_k = torch_mod.zeros((h + 1, w + 7), dtype=torch_mod.uint8, device="cuda")
    m = big_m[:, 1:1 + w]
    k = big_k[1:, 3:3 + w]
    m.copy_(torch_mod.from_numpy(marker))
    k.copy_(torch_mod.from_numpy(mask))
    rc.erode(m, k, 8)
    rc.last_stats()
    assert_same(m.cpu().numpy(), oracle_mod.recon_erode(marker, mask, 8), "erode, unaligned views")
    assert int(big_m[:, 0].sum()) == 0 and int(big_m[:, 1 + w:].sum()) == 0
    assert_same(k.cpu().numpy(), mask, "the mask is not written")
    # h-dome and regional maxima in place on an offset view with a padded pitch
    for op in ("hdome", "regional_max"):
        big = torch_mod.zeros((h + 2, w + 9), dtype=torch_mod.uint8, device="cuda")
        v = big[1:1 + h, 2:2 + w]
        v.copy_(torch_mod.from_numpy(mask))
        if op == "hdome":
            rc.hdome(v, 40, 4)
            want = oracle_mod.hdome(mask, 40, 4)
        else:
            rc.regional_max(v, 4)
            want = oracle_mod.regional_max(mask, 4)
        rc.last_stats()
        assert_same(v.cpu().numpy(), want, "%s, unaligned view" % op)
        assert int(big[0].sum()) == 0 and int(big[:, :2].sum()) == 0 and int(big[:, 2 + w:].sum()) == 0


def _mixed_tasks(rng, n):
    ops = ["dilate", "fill_holes", "erode", "hdome", "regional_max"]
    tasks = []
    for i in range(n):
        hh, ww = int(rng.integers(1, 600)), int(rng.integers(1, 800))
        conn = int(rng.choice([4, 8]))
        mask = synth.scaled_config1_tile(hh, ww, 9000 + i)
        op = ops[i % len(ops)]
        if op == "dilate":
            tasks.append({"op": op, "marker": synth.hdome_marker(mask, 20), "mask": mask, "conn": conn})
        elif op == "erode":
            tasks.append({"op": op, "marker": raised(mask, 20), "mask": mask, "conn": conn})
        elif op == "fill_holes":
            tasks.append({"op": op, "img": np.where(mask > 60, 255, 0).astype(np.uint8), "conn": conn})
        elif op == "hdome":
            tasks.append({"op": op, "img": mask, "h": int(rng.integers(1, 256)), "conn": conn})
        else:
            tasks.append({"op": op, "img": mask, "conn": conn})
    return tasks


def _run_batch(torch_mod, ctx, tasks):
    devs, spec = [], []
    for t in tasks:
        if t["op"] in ("dilate", "erode"):
            m, k = dev(torch_mod, t["marker"]), dev(torch_mod, t["mask"])
            devs.append(m)
            spec.append({"op": t["op"], "image": m, "mask": k, "conn": t["conn"]})
        else:
            x = dev(torch_mod, t["img"])
            devs.append(x)
            spec.append({"op": t["op"], "image": x, "conn": t["conn"], "h": t.get("h", 0)})
    ctx.batch(spec)
    ctx.last_stats()
    return [d.cpu().numpy() for d in devs]


def test_batch_of_all_ops(torch_mod, rc, oracle_mod):
    # more tasks than travel in the kernel arguments, then a replay of the
    # captured graph with a different (smaller) batch
    for seed, n in ((501, 17), (502, 13)):
        tasks = _mixed_tasks(np.random.default_rng(seed), n)
        outs = _run_batch(torch_mod, rc, tasks)
        for i, (t, got) in enumerate(zip(tasks, outs)):
            assert_same(got, oracle_mod.run_task(t), "batch %d task %d (%s)" % (seed, i, t["op"]))


def test_serving_all_ops(torch_mod, lib, oracle_mod):
    tasks = _mixed_tasks(np.random.default_rng(503), 10)
    with lib.Recon(0) as ctx:
        held = []
        for t in tasks:
            if t["op"] in ("dilate", "erode"):
                m, k = dev(torch_mod, t["marker"]), dev(torch_mod, t["mask"])
                torch_mod.cuda.synchronize()
                tk = ctx.submit(t["op"], m, k, conn=t["conn"])
            else:
                m = dev(torch_mod, t["img"])
                torch_mod.cuda.synchronize()
                tk = ctx.submit(t["op"], m, conn=t["conn"], h=t.get("h", 0))
            held.append((tk, m))
        for i, ((tk, m), t) in enumerate(zip(held, tasks)):
            ctx.wait(tk, 60_000_000)
            assert_same(m.cpu().numpy(), oracle_mod.run_task(t), "served task %d (%s)" % (i, t["op"]))
        ctx.serve_stop()


@pytest.mark.parametrize("cfg", [dict(block_rows=16), dict(block_rows=64), dict(queue_capacity=64),
                                 dict(scan_rounds=-1), dict(stop_after_stage=3),
                                 dict(drain_budget=1, binary_drain_budget=1)], ids=str)
def test_tuning_invariance(torch_mod, lib, oracle_mod, cfg):
    _, mask, _ = synth.config2_tile(seed=synth.seed_for(2, 13), size=768, n_gauss=106)
    up = raised(mask, 30)
    with lib.Recon(0, **cfg) as ctx:
        for conn in (8, 4):
            assert_same(gpu_erode(torch_mod, ctx, up, mask, conn), oracle_mod.recon_erode(up, mask, conn),
                        "%s erode conn %d" % (cfg, conn))
            assert_same(gpu_hdome(torch_mod, ctx, mask, 30, conn), oracle_mod.hdome(mask, 30, conn),
                        "%s hdome conn %d" % (cfg, conn))
            assert_same(gpu_rmax(torch_mod, ctx, mask, conn), oracle_mod.regional_max(mask, conn),
                        "%s regional max conn %d" % (cfg, conn))


def test_argument_errors(torch_mod, rc, lib):
    a = torch_mod.zeros((4, 5), dtype=torch_mod.uint8, device="cuda")
    b = torch_mod.zeros((4, 6), dtype=torch_mod.uint8, device="cuda")
    c = torch_mod.zeros((4, 5), dtype=torch_mod.uint8, device="cuda")
    with pytest.raises(lib.ReconError):
        rc.erode(a, b, 8)          # shapes differ
    with pytest.raises(lib.ReconError):
        rc.erode(a, a, 8)          # marker and mask overlap
    with pytest.raises(lib.ReconError):
        rc.erode(a, c, 6)
    for h in (0, 256, -1):
        with pytest.raises(lib.ReconError):
            rc.hdome(a, h, 8)
    with pytest.raises(lib.ReconError):
        rc.regional_max(a, 5)
    with pytest.raises(ValueError):
        lib.make_task("opening", a)
    # nothing was enqueued: a valid call still works afterwards
    rc.regional_max(a, 8)
    rc.last_stats()
    assert int(a.sum()) == 0
