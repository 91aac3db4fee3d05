"""GPU parity: the HIP path through the C ABI must equal the CPU oracle byte for byte.

All inputs are seeded and synthetic.  Integer work, so the bar is bit-exact
(tolerance 0) everywhere: every tile shape, connectivity, tuning, batch mix
and repetition.
"""
import numpy as np
import pytest

import golden_io
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


def gpu_dilate(torch_mod, ctx, marker, mask, conn):
    m = dev(torch_mod, marker)
    k = dev(torch_mod, mask)
    ctx.dilate(m, k, conn)
    ctx.last_stats()  # waits with a deadline; raises if the launch timed out or was stopped
    return m.cpu().numpy()


def gpu_fill(torch_mod, ctx, img, conn):
    x = dev(torch_mod, img)
    ctx.fill_holes(x, conn)
    ctx.last_stats()
    return x.cpu().numpy()


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("%s: %d pixels differ, first at (%d, %d): got %d want %d"
                             % (what, len(bad), y, x, got[y, x], want[y, x]))


def test_context_self_test(lib, torch_mod):
    # context creation runs the library's self-test kernel (with a deadline)
    with lib.Recon(0) as ctx:
        assert ctx.ctx


def _blockwise(oracle_mod, marker, mask, conn, bh=32, bw=256):
    want = np.empty_like(mask)
    for y0 in range(0, mask.shape[0], bh):
        for x0 in range(0, mask.shape[1], bw):
            sl = np.s_[y0:y0 + bh, x0:x0 + bw]
            want[sl] = oracle_mod.recon_dilate(marker[sl], mask[sl], conn)
    return want


@pytest.mark.parametrize("conn", [8, 4])
def test_stage1_dense_pass_blockwise(torch_mod, lib, oracle_mod, conn):
    # the first kernel alone reconstructs every 32 x 256 block on its own
    rng = np.random.default_rng(50 + conn)
    mask = rng.integers(0, 256, (70, 600)).astype(np.uint8)
    marker = synth.hdome_marker(mask, 50)
    c1m, c1k = synth.config1_tile()
    with lib.Recon(0, stop_after_stage=1) as ctx:
        for m, k in ((marker, mask), (c1m, c1k)):
            assert_same(gpu_dilate(torch_mod, ctx, m, k, conn), _blockwise(oracle_mod, m, k, conn),
                        "dense pass %s conn %d" % (k.shape, conn))


@pytest.mark.parametrize("case", golden_io.all_cases(), ids=lambda c: c["name"])
def test_golden(torch_mod, rc, case):
    for conn in case["conns"]:
        if case["op"] == "dilate":
            got = gpu_dilate(torch_mod, rc, case["marker"], case["mask"], conn)
        else:
            got = gpu_fill(torch_mod, rc, case["img"], conn)
        assert_same(got, case["expect"], "%s conn %d" % (case["name"], conn))


@pytest.mark.parametrize("conn", [8, 4])
def test_config1_tile(torch_mod, rc, oracle_mod, conn):
    marker, mask = synth.config1_tile()
    assert_same(gpu_dilate(torch_mod, rc, marker, mask, conn), oracle_mod.recon_dilate(marker, mask, conn),
                "512x512 nuclei conn %d" % conn)


SHAPES = [(1, 1), (1, 7), (7, 1), (1, 300), (300, 1), (2, 2), (3, 257), (65, 3), (31, 256), (32, 256),
          (33, 257), (64, 512), (257, 131), (100, 513), (129, 1000)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
@pytest.mark.parametrize("conn", [8, 4])
def test_ragged_shapes(torch_mod, rc, oracle_mod, shape, conn):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1] + conn)
    for levels in (3, 256):
        marker, mask = synth.random_pair(rng, shape[0], shape[1], levels)
        if levels == 256:
            marker = synth.hdome_marker(mask, int(rng.integers(1, 80)))
        assert_same(gpu_dilate(torch_mod, rc, marker, mask, conn), oracle_mod.recon_dilate(marker, mask, conn),
                    "%dx%d levels %d conn %d" % (shape[0], shape[1], levels, conn))


@pytest.mark.parametrize("conn", [8, 4])
def test_marker_above_mask_is_clipped(torch_mod, rc, oracle_mod, conn):
    rng = np.random.default_rng(9)
    marker, mask = synth.random_pair(rng, 70, 300, 256)
    assert_same(gpu_dilate(torch_mod, rc, marker, mask, conn), oracle_mod.recon_dilate(marker, mask, conn),
                "unclipped marker")


@pytest.mark.parametrize("conn", [8, 4])
def test_nuclei_1024(torch_mod, rc, oracle_mod, conn):
    marker, mask, binary = synth.config2_tile(seed=synth.seed_for(2, 7), size=1024, n_gauss=188)
    assert_same(gpu_dilate(torch_mod, rc, marker, mask, conn), oracle_mod.recon_dilate(marker, mask, conn),
                "1024 nuclei conn %d" % conn)
    assert_same(gpu_fill(torch_mod, rc, binary, conn), oracle_mod.fill_holes(binary, conn),
                "1024 fill conn %d" % conn)


@pytest.mark.parametrize("conn", [8, 4])
def test_config2_full_tile(torch_mod, rc, oracle_mod, conn):
    marker, mask, binary = synth.config2_tile()
    assert_same(gpu_dilate(torch_mod, rc, marker, mask, conn), oracle_mod.recon_dilate(marker, mask, conn),
                "4096 nuclei conn %d" % conn)
    assert_same(gpu_fill(torch_mod, rc, binary, conn), oracle_mod.fill_holes(binary, conn),
                "4096 fill conn %d" % conn)


@pytest.mark.parametrize("conn", [8, 4])
def test_fill_holes_grey_and_ragged(torch_mod, rc, oracle_mod, conn):
    rng = np.random.default_rng(31 + conn)
    for shape in [(1, 1), (2, 5), (5, 2), (3, 3), (40, 300), (257, 131)]:
        img = rng.integers(0, 256, size=shape).astype(np.uint8)
        assert_same(gpu_fill(torch_mod, rc, img, conn), oracle_mod.fill_holes(img, conn), "grey fill %s" % (shape,))
        b = np.where(rng.random(shape) < 0.55, 255, 0).astype(np.uint8)
        assert_same(gpu_fill(torch_mod, rc, b, conn), oracle_mod.fill_holes(b, conn), "binary fill %s" % (shape,))


@pytest.mark.parametrize("route", [0, -1], ids=["component", "block"])
@pytest.mark.parametrize("seed_at", ["outer", "inner"])
def test_spiral_1024(torch_mod, lib, seed_at, route):
    # both routes: labelling (the default for a two-valued mask) and block visits
    marker, mask, _ = synth.spiral_tile(1024, 1024, seed_at)
    with lib.Recon(0, component_route=route) as ctx:
        for conn in (8, 4):
            assert_same(gpu_dilate(torch_mod, ctx, marker, mask, conn), mask,
                        "spiral %s conn %d route %d" % (seed_at, conn, route))


def test_unaligned_pitch_and_offset(torch_mod, rc, oracle_mod):
    rng = np.random.default_rng(4)
    h, w = 90, 301
    marker, mask = synth.random_pair(rng, h, w, 256)
    marker = synth.hdome_marker(mask, 25)
    big_m = torch_mod.zeros((h, w + 7), dtype=torch_mod.uint8, device="cuda")
    big_k = torch_mod.zeros((h + 1, w + 7), dtype=torch_mod.uint8, device="cuda")
    m = big_m[:, 1:1 + w]
    k = big_k[1:, 3:3 + w]
    m.copy_(torch_mod.from_numpy(marker))
    k.copy_(torch_mod.from_numpy(mask))
    rc.dilate(m, k, 8)
    rc.last_stats()
    assert_same(m.cpu().numpy(), oracle_mod.recon_dilate(marker, mask, 8), "unaligned views")
    # the padding around the views is untouched
    assert int(big_m[:, 0].sum()) == 0 and int(big_m[:, 1 + w:].sum()) == 0


@pytest.mark.parametrize("cfg", [dict(block_rows=16), dict(block_rows=64), dict(queue_capacity=64),
                                 dict(queue_capacity=64, spill_capacity=-1), dict(queue_capacity=64, spill_capacity=64),
                                 dict(scan_rounds=-1), dict(scan_rounds=4, block_rows=64),
                                 dict(wg_per_cu=1), dict(stop_after_stage=3),
                                 dict(drain_budget=1, binary_drain_budget=1),
                                 dict(drain_budget=4096, binary_drain_budget=4096)], ids=str)
def test_tuning_invariance(torch_mod, lib, oracle_mod, cfg):
    marker, mask, binary = synth.config2_tile(seed=synth.seed_for(2, 11), size=768, n_gauss=106)
    sm, smask, _ = synth.spiral_tile(300, 520, "inner")
    # the binary fill and the spiral take the block route too (component_route -1)
    for route in (0, -1):
        with lib.Recon(0, component_route=route, **cfg) as ctx:
            for conn in (8, 4):
                what = "%s conn %d route %d" % (cfg, conn, route)
                assert_same(gpu_dilate(torch_mod, ctx, marker, mask, conn),
                            oracle_mod.recon_dilate(marker, mask, conn), what)
                assert_same(gpu_fill(torch_mod, ctx, binary, conn), oracle_mod.fill_holes(binary, conn),
                            "fill " + what)
                assert_same(gpu_dilate(torch_mod, ctx, sm, smask, conn), smask, "spiral " + what)


def test_determinism(torch_mod, rc):
    marker, mask, _ = synth.config2_tile(seed=synth.seed_for(2, 12), size=1024, n_gauss=188)
    first = gpu_dilate(torch_mod, rc, marker, mask, 8)
    for _ in range(5):
        assert np.array_equal(gpu_dilate(torch_mod, rc, marker, mask, 8), first)


def _batch_tasks(rng, n):
    tasks = []
    for i in range(n):
        h, w = int(rng.integers(1, 700)), int(rng.integers(1, 900))
        conn = int(rng.choice([4, 8]))
        if i % 5 == 4:
            img = np.where(rng.random((h, w)) < 0.6, 255, 0).astype(np.uint8)
            tasks.append({"op": "fill_holes", "img": img, "conn": conn})
        else:
            mask = synth.scaled_config1_tile(h, w, 5000 + i)
            tasks.append({"op": "dilate", "marker": synth.hdome_marker(mask, int(rng.integers(10, 41))),
                          "mask": mask, "conn": conn})
    return tasks


def _run_batch(torch_mod, ctx, tasks):
    devs = []
    spec = []
    for t in tasks:
        if t["op"] == "dilate":
            m, k = dev(torch_mod, t["marker"]), dev(torch_mod, t["mask"])
            devs.append(m)
            spec.append({"op": "dilate", "image": m, "mask": k, "conn": t["conn"]})
        else:
            x = dev(torch_mod, t["img"])
            devs.append(x)
            spec.append({"op": "fill_holes", "image": x, "conn": t["conn"]})
    ctx.batch(spec)
    ctx.last_stats()
    return [d.cpu().numpy() for d in devs]


def test_batch_mixed(torch_mod, rc, oracle_mod):
    rng = np.random.default_rng(123)
    tasks = _batch_tasks(rng, 23)
    outs = _run_batch(torch_mod, rc, tasks)
    for i, (t, got) in enumerate(zip(tasks, outs)):
        assert_same(got, oracle_mod.run_task(t), "batch task %d (%s)" % (i, t["op"]))
    # replay of the captured graph with a different batch (more than the 12
    # tasks a direct launch takes in its arguments)
    tasks2 = _batch_tasks(np.random.default_rng(321), 13)
    outs2 = _run_batch(torch_mod, rc, tasks2)
    for i, (t, got) in enumerate(zip(tasks2, outs2)):
        assert_same(got, oracle_mod.run_task(t), "second batch task %d" % i)


def test_batch_with_spirals(torch_mod, rc, oracle_mod):
    tasks = synth.config3_batch(n_tiles=8, size=512)
    outs = _run_batch(torch_mod, rc, tasks)
    for i, (t, got) in enumerate(zip(tasks, outs)):
        assert_same(got, oracle_mod.run_task(t), "config-3 style task %d (%s)" % (i, t["kind"]))


def test_graph_replays_with_timing(torch_mod, lib, oracle_mod):
    """The same batch replayed from the captured graph three times, with eager
    work and synchronisation in between, equals the plain per-task calls each
    time; timing a graph replay reports the launch total only and leaves no HIP
    error behind for the next torch call."""
    rng = np.random.default_rng(77)
    tasks = _batch_tasks(rng, 14)
    with lib.Recon(0, timing=1) as ctx:
        eager = []
        for t in tasks:
            if t["op"] == "dilate":
                eager.append(gpu_dilate(torch_mod, ctx, t["marker"], t["mask"], t["conn"]))
            else:
                eager.append(gpu_fill(torch_mod, ctx, t["img"], t["conn"]))
        for rep in range(3):
            outs = _run_batch(torch_mod, ctx, tasks)
            st = ctx.last_stats()
            assert st["total_ms"] > 0 and st["dense_ms"] == -1.0
            probe = torch_mod.arange(1000, device="cuda").sum().item()   # eager work in between
            assert probe == 499500
            torch_mod.cuda.synchronize()
            for i, (want, got) in enumerate(zip(eager, outs)):
                assert_same(got, want, "replay %d task %d" % (rep, i))
    for i, (t, got) in enumerate(zip(tasks, eager)):
        assert_same(got, oracle_mod.run_task(t), "eager task %d" % i)


def test_argument_errors(torch_mod, rc, lib):
    a = torch_mod.zeros((4, 5), dtype=torch_mod.uint8, device="cuda")
    b = torch_mod.zeros((4, 6), dtype=torch_mod.uint8, device="cuda")
    with pytest.raises(lib.ReconError):
        rc.dilate(a, b, 8)
    c = torch_mod.zeros((4, 5), dtype=torch_mod.uint8, device="cuda")
    with pytest.raises(lib.ReconError):
        rc.dilate(a, c, 6)
    with pytest.raises(lib.ReconError):
        rc.dilate(a, a, 8)  # marker and mask overlap
    with pytest.raises(lib.ReconError):
        rc.fill_holes(a, 5)


def test_small_batch_in_timing_context(torch_mod, lib, oracle_mod):
    """A batch of at most 12 tasks is launched directly: in a timing context
    every kernel is timed, and the bytes equal the oracle's (the headline step
    runs a tile's reconstruction and fill-holes this way)."""
    marker, mask, binary = synth.config2_tile(seed=synth.seed_for(2, 14), size=1024, n_gauss=188)
    with lib.Recon(0, timing=1) as ctx:
        for rep in range(2):
            m, k, b = dev(torch_mod, marker), dev(torch_mod, mask), dev(torch_mod, binary)
            ctx.batch([{"op": "dilate", "image": m, "mask": k, "conn": 8},
                       {"op": "fill_holes", "image": b, "conn": 8}])
            st = ctx.last_stats()
            assert st["drain_ms"] > 0 and st["total_ms"] >= st["drain_ms"]
            # beside the grey reconstruction the binary fill-holes (thick
            # foreground) keeps the block route: both tasks' 32 x 4 blocks are visited
            assert st["dense_visits"] == 2 * 32 * 4 and st["component_tasks"] == 0
            t = ctx.launch_times(0)
            assert t["drain_ms"] == st["drain_ms"]
            assert_same(m.cpu().numpy(), oracle_mod.recon_dilate(marker, mask, 8), "batched dilate %d" % rep)
            assert_same(b.cpu().numpy(), oracle_mod.fill_holes(binary, 8), "batched fill %d" % rep)


def test_max_size_tile(torch_mod, rc, oracle_mod):
    """The largest tile of the tests: 16384 x 16384 (268 Mpx per plane, 65536
    blocks), the nuclei generator scaled to its area; reconstruction and
    fill-holes compared with the oracle over the whole tile."""
    mask = synth.scaled_config1_tile(16384, 16384, synth.seed_for(6, 0))
    marker = synth.hdome_marker(mask, 30)
    assert_same(gpu_dilate(torch_mod, rc, marker, mask, 8), oracle_mod.recon_dilate(marker, mask, 8),
                "16384 nuclei dilate")
    binary = np.where(mask > 120, 255, 0).astype(np.uint8)
    assert_same(gpu_fill(torch_mod, rc, binary, 8), oracle_mod.fill_holes(binary, 8), "16384 fill")


def test_failed_claims_report_edevice(torch_mod, lib):
    """A launch whose block claims keep failing gives up (every wave leaves)
    and the host reports RECON_EDEVICE instead of a silently wrong result.
    The context's test hook makes every claim's compare-and-swap fail."""
    mask = synth.gaussian_tile(100, 300, 5, seed=3)
    with lib.Recon(0, test_fault=1) as ctx:
        m = dev(torch_mod, synth.hdome_marker(mask, 30))
        ctx.dilate(m, dev(torch_mod, mask), 8)
        with pytest.raises(lib.ReconError) as e:
            ctx.last_stats()
        assert e.value.code == lib.RECON_EDEVICE


def test_spill_queue_takes_the_overflow(torch_mod, lib, oracle_mod):
    """With a 64-entry LDS queue, pushes that do not fit go to the wave's
    global spill queue, and the block re-seeds only when that is full too;
    without the spill every LDS overflow re-seeds.  Bytes equal the oracle's
    both ways."""
    marker, mask, _ = synth.config2_tile(seed=synth.seed_for(2, 42), size=1024, n_gauss=188)
    want = oracle_mod.recon_dilate(marker, mask, 4)
    seen = {}
    for spill in (0, -1):
        with lib.Recon(0, queue_capacity=64, scan_rounds=-1, spill_capacity=spill) as ctx:
            m, k = dev(torch_mod, marker), dev(torch_mod, mask)
            ctx.dilate(m, k, 4)
            seen[spill] = ctx.last_stats()
            assert_same(m.cpu().numpy(), want, "queue 64, spill %d" % spill)
    assert seen[0]["queue_spills"] > 0, seen[0]
    assert seen[-1]["queue_spills"] == 0 and seen[-1]["queue_overflows"] > 0, seen[-1]
    assert seen[0]["queue_overflows"] < seen[-1]["queue_overflows"], (seen[0], seen[-1])
