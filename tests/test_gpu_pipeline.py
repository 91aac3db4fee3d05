"""GPU parity of the co-scheduled tile pipeline (recon_pipeline_run) through
the C ABI: the GPU alone and the GPU beside CPU workers, under FCFS and PATS,
with and without data locality, at several window sizes.  Wherever each
operation instance runs, every tile's outputs must equal the oracle's
composition of the same operations (integer work: tolerance 0).  Inputs are
seeded synthetic nuclei-like tiles of several shapes (ragged ones included)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

H, LO, HI = 20, 20, 1000


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


@pytest.fixture(scope="module")
def tiles():
    rng = np.random.default_rng(31)
    return [synth.scaled_config1_tile(512, 512, synth.seed_for(9, 20)),
            synth.scaled_config1_tile(300, 410, synth.seed_for(9, 21)),
            synth.scaled_config1_tile(777, 259, synth.seed_for(9, 22)),
            rng.integers(0, 256, size=(1, 97), dtype=np.uint8),
            synth.scaled_config1_tile(256, 1024, synth.seed_for(9, 23)),
            np.zeros((19, 5), np.uint8),
            synth.scaled_config1_tile(640, 480, synth.seed_for(9, 24))]


@pytest.fixture(scope="module")
def expected(tiles, oracle_mod):
    out = {}
    for conn in (4, 8):
        res = []
        for img in tiles:
            d = oracle_mod.hdome(img, H, conn)
            f = oracle_mod.fill_holes(d, conn)
            a = oracle_mod.area_threshold(f, LO, HI, conn)
            lab, n = oracle_mod.label(a, conn)
            res.append({"objects": a, "markers": oracle_mod.pre_watershed(a, conn), "labels": lab, "count": n})
        out[conn] = res
    return out


def check(outs, want):
    for i, (o, w) in enumerate(zip(outs, want)):
        for k in ("objects", "markers", "labels"):
            assert np.array_equal(o[k], w[k]), (i, k, int((o[k] != w[k]).sum()))
        assert o["count"] == w["count"], i


SPEEDUP = {"hdome": 40.0, "fill_holes": 60.0, "area_threshold": 8.0, "markers": 25.0, "label": 3.0}


@pytest.mark.parametrize("conn", [4, 8])
def test_gpu_only(lib, rc, tiles, expected, conn):
    cfg = lib.pipe_config(policy="pats", cpu_workers=0, use_gpu=True, window=3, conn=conn, h=H,
                          area_min=LO, area_max=HI)
    outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg)
    check(outs, expected[conn])
    assert st["ops_gpu"] == [len(tiles)] * 5 and st["ops_cpu"] == [0] * 5
    # data locality: the image goes up once and the three results come back once
    assert st["uploads"] == len(tiles) and st["downloads"] == 3 * len(tiles)


@pytest.mark.parametrize("policy", ["fcfs", "pats"])
@pytest.mark.parametrize("dl", [True, False])
@pytest.mark.parametrize("window", [1, 4])
def test_gpu_and_cpu_workers(lib, rc, tiles, expected, policy, dl, window):
    cfg = lib.pipe_config(policy=policy, cpu_workers=3, use_gpu=True, window=window, data_locality=dl,
                          conn=8, h=H, area_min=LO, area_max=HI, speedup=SPEEDUP,
                          transfer_impact={"label": 0.5, "markers": 0.2})
    outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg)
    check(outs, expected[8])
    assert [a + b for a, b in zip(st["ops_cpu"], st["ops_gpu"])] == [len(tiles)] * 5
    if not dl:
        # the basic mode moves every GPU assignment's inputs in and outputs out
        assert st["uploads"] >= sum(st["ops_gpu"])


@pytest.mark.parametrize("cpu_workers", [0, 3])
def test_prefetch(lib, rc, tiles, expected, cpu_workers):
    """Prefetching uploads each admitted image before its first operation:
    the same bytes, and with the GPU alone one upload per tile, none on demand."""
    cfg = lib.pipe_config(policy="pats", cpu_workers=cpu_workers, use_gpu=True, window=2, conn=8, h=H,
                          area_min=LO, area_max=HI, speedup=SPEEDUP, prefetch=True)
    outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg)
    check(outs, expected[8])
    if cpu_workers == 0:
        assert st["uploads"] == len(tiles) and st["downloads"] == 3 * len(tiles)


@pytest.mark.parametrize("policy", ["fcfs", "pats"])
def test_cpu_limits(lib, rc, tiles, expected, policy):
    """The CPU cut-off and the remaining-work guard change who runs what, never the bytes."""
    gpu_ms = {"hdome": 0.5, "fill_holes": 0.5, "area_threshold": 0.2, "markers": 0.3, "label": 0.1}
    for kw in (dict(cpu_max_speedup=10.0), dict(cpu_guard=True, gpu_ms=gpu_ms),
               dict(cpu_max_speedup=30.0, cpu_guard=True, gpu_ms=gpu_ms)):
        cfg = lib.pipe_config(policy=policy, cpu_workers=3, use_gpu=True, window=4, conn=8, h=H, area_min=LO,
                              area_max=HI, speedup=SPEEDUP, **kw)
        outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg)
        check(outs, expected[8])
        if "cpu_max_speedup" in kw:
            # the workers never take an operation whose estimate is above the limit
            for k, op in enumerate(lib.PIPE_OPS):
                if SPEEDUP[op] > kw["cpu_max_speedup"]:
                    assert st["ops_cpu"][k] == 0, (kw, op)


ORDER_SPEEDUP = {"hdome": 30, "fill_holes": 20, "area_threshold": 5, "markers": 10, "label": 2}
SHORT = {"hdome": "h", "fill_holes": "f", "area_threshold": "a", "markers": "m", "label": "l"}


@pytest.mark.parametrize("policy,dl,impact,want", [
    # PATS on the GPU: the highest estimated speedup first
    ("pats", False, 0.0, "h0 h1 h2 f0 f1 f2 a0 m0 a1 m1 a2 m2 l0 l1 l2"),
    # data locality with PATS: a resident instance wins when its speedup is at
    # least the best one's times (1 - transfer impact of the best one's operation)
    ("pats", True, 0.0, "h0 h1 h2 f0 f1 f2 a0 m0 a1 m1 a2 m2 l0 l1 l2"),
    ("pats", True, 0.5, "h0 f0 h1 f1 h2 f2 a0 m0 a1 m1 a2 m2 l0 l1 l2"),
    # FCFS with data locality always prefers resident data (oldest first)
    ("fcfs", True, 0.0, "h0 f0 a0 m0 l0 h1 f1 a1 m1 l1 h2 f2 a2 m2 l2"),
    ("fcfs", False, 0.0, "h0 h1 h2 f0 f1 f2 a0 a1 a2 m0 l0 m1 l1 m2 l2"),
])
def test_policy_order_on_the_gpu(lib, rc, policy, dl, impact, want):
    """With the GPU alone the order of the instances is fixed by the policy and
    the data-locality rule; the trace must show exactly the rule."""
    tiles = [synth.scaled_config1_tile(64, 96, synth.seed_for(9, 40 + i)) for i in range(3)]
    cfg = lib.pipe_config(policy=policy, cpu_workers=0, use_gpu=True, window=3, data_locality=dl,
                          speedup=ORDER_SPEEDUP, transfer_impact={k: impact for k in ORDER_SPEEDUP})
    _, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg, trace=True)
    got = " ".join("%s%d" % (SHORT[op], tile) for tile, op, dev, t0, t1 in st["trace"])
    assert got == want
    assert all(dev == 0 for _, _, dev, _, _ in st["trace"])


def test_pipeline_twice_in_a_row_and_after_other_work(lib, rc, tiles, expected, torch_mod):
    cfg = lib.pipe_config(policy="pats", cpu_workers=2, use_gpu=True, window=2, conn=8, h=H,
                          area_min=LO, area_max=HI, speedup=SPEEDUP)
    outs1, _ = lib.recon_pipeline_run(rc.ctx, tiles[:3], cfg)
    # the context keeps serving ordinary calls between pipeline runs
    m = torch_mod.from_numpy(tiles[0]).cuda()
    rc.hdome(m, H, 8)
    torch_mod.cuda.synchronize()
    outs2, _ = lib.recon_pipeline_run(rc.ctx, tiles[2:], cfg)
    check(outs1, expected[8][:3])
    check(outs2, expected[8][2:])


def test_pipeline_full_size_tiles(lib, rc, oracle_mod):
    """Two 4096 x 4096 nuclei-like tiles (the benchmark's tile size) through
    the pipeline with CPU workers under PATS with the remaining-work guard,
    against the oracle's chain."""
    tiles = [synth.config2_tile(seed=synth.seed_for(6, 900 + i))[1] for i in range(2)]
    gpu_ms = {"hdome": 1.5, "fill_holes": 2.0, "area_threshold": 0.6, "markers": 0.8, "label": 0.4}
    speed = {"hdome": 450.0, "fill_holes": 200.0, "area_threshold": 240.0, "markers": 260.0, "label": 200.0}
    cfg = lib.pipe_config(policy="pats", cpu_workers=4, use_gpu=True, window=2, conn=8, h=H, area_min=LO,
                          area_max=HI, speedup=speed, gpu_ms=gpu_ms, cpu_guard=True)
    outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg)
    want = []
    for img in tiles:
        a = oracle_mod.area_threshold(oracle_mod.fill_holes(oracle_mod.hdome(img, H, 8), 8), LO, HI, 8)
        lab, n = oracle_mod.label(a, 8)
        want.append({"objects": a, "markers": oracle_mod.pre_watershed(a, 8), "labels": lab, "count": n})
    check(outs, want)
    assert [a + b for a, b in zip(st["ops_cpu"], st["ops_gpu"])] == [2] * 5


def test_many_workers_and_io_threads(lib, rc, oracle_mod):
    """Twelve CPU workers, four I/O threads, prefetching, a window of 6 over 16
    tiles of mixed shapes, both policies with data locality and the guard, with
    the trace on: every instance runs once, and every tile equals the oracle's chain."""
    tiles = [synth.scaled_config1_tile(96 + 37 * (i % 5), 160 + 61 * (i % 3), synth.seed_for(9, 70 + i))
             for i in range(16)]
    want = []
    for img in tiles:
        a = oracle_mod.area_threshold(oracle_mod.fill_holes(oracle_mod.hdome(img, H, 8), 8), LO, HI, 8)
        lab, n = oracle_mod.label(a, 8)
        want.append({"objects": a, "markers": oracle_mod.pre_watershed(a, 8), "labels": lab, "count": n})
    gpu_ms = {"hdome": 0.2, "fill_holes": 0.2, "area_threshold": 0.1, "markers": 0.1, "label": 0.05}
    for policy in ("fcfs", "pats"):
        cfg = lib.pipe_config(policy=policy, cpu_workers=12, use_gpu=True, window=6, data_locality=True, conn=8,
                              h=H, area_min=LO, area_max=HI, speedup=SPEEDUP, io_threads=4, prefetch=True,
                              gpu_ms=gpu_ms, cpu_guard=(policy == "pats"))
        outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg, trace=True)
        check(outs, want)
        seen = sorted((t, op) for t, op, _, _, _ in st["trace"])
        assert seen == sorted((t, op) for t in range(16) for op in lib.PIPE_OPS)


@pytest.mark.parametrize("depth", [2, 3])
@pytest.mark.parametrize("cpu_workers,policy,dl,prefetch", [(0, "pats", True, True), (0, "fcfs", False, False),
                                                            (3, "pats", True, False), (3, "fcfs", False, True)])
def test_gpu_inflight(lib, rc, tiles, expected, depth, cpu_workers, policy, dl, prefetch):
    """The GPU manager with 2 or 3 instances enqueued on its stream at once,
    alone or beside CPU workers, with and without data locality: every tile
    equals the oracle's chain and every instance runs once."""
    gpu_ms = {"hdome": 0.2, "fill_holes": 0.2, "area_threshold": 0.1, "markers": 0.1, "label": 0.05}
    cfg = lib.pipe_config(policy=policy, cpu_workers=cpu_workers, use_gpu=True, window=4, data_locality=dl,
                          conn=8, h=H, area_min=LO, area_max=HI, speedup=SPEEDUP, gpu_ms=gpu_ms,
                          cpu_guard=cpu_workers > 0, prefetch=prefetch, gpu_inflight=depth)
    outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg, trace=True)
    check(outs, expected[8])
    assert [a + b for a, b in zip(st["ops_cpu"], st["ops_gpu"])] == [len(tiles)] * 5
    seen = sorted((t, op) for t, op, _, _, _ in st["trace"])
    assert seen == sorted((t, op) for t in range(len(tiles)) for op in lib.PIPE_OPS)
    if cpu_workers == 0 and dl:
        assert st["uploads"] == len(tiles) and st["downloads"] == 3 * len(tiles)


def test_gpu_inflight_full_size_tiles(lib, rc, oracle_mod):
    """Five 4096 x 4096 nuclei-like tiles with two instances in flight on the
    GPU and prefetching, against the oracle's chain."""
    tiles = [synth.config2_tile(seed=synth.seed_for(6, 960 + i))[1] for i in range(5)]
    cfg = lib.pipe_config(policy="pats", cpu_workers=0, use_gpu=True, window=3, conn=8, h=H, area_min=LO,
                          area_max=HI, speedup=SPEEDUP, prefetch=True, io_threads=4, gpu_inflight=2)
    outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg)
    for img, o in zip(tiles, outs):
        a = oracle_mod.area_threshold(oracle_mod.fill_holes(oracle_mod.hdome(img, H, 8), 8), LO, HI, 8)
        lab, n = oracle_mod.label(a, 8)
        assert np.array_equal(o["objects"], a) and np.array_equal(o["markers"], oracle_mod.pre_watershed(a, 8))
        assert np.array_equal(o["labels"], lab) and o["count"] == n
    assert st["ops_gpu"] == [5] * 5


def test_enqueue_status(lib, torch_mod):
    """recon_enqueue_status writes 0 after a launch that converged (and before
    any launch), 1 after one its scheduler gave up (the context's test hook
    makes every block claim fail), into pinned host memory, without a wait."""
    mask = synth.gaussian_tile(100, 300, 5, seed=3)
    flag = torch_mod.full((4,), 7, dtype=torch_mod.int32).pin_memory()
    stream = torch_mod.cuda.current_stream()
    for fault, want in ((0, 0), (1, 1)):
        with lib.Recon(0, test_fault=fault) as ctx:
            lib.recon_enqueue_status(ctx.ctx, flag.data_ptr() + 4, stream)   # no launch yet
            m = torch_mod.from_numpy(synth.hdome_marker(mask, 30)).cuda()
            ctx.dilate(m, torch_mod.from_numpy(mask).cuda(), 8, stream)
            lib.recon_enqueue_status(ctx.ctx, flag.data_ptr(), stream)
            torch_mod.cuda.synchronize()
            assert int(flag[0]) == want and int(flag[1]) == 0, (fault, flag.tolist())
            if fault:
                with pytest.raises(lib.ReconError):
                    ctx.last_stats()


@pytest.mark.parametrize("batch,depth", [(4, 1), (8, 2)])
@pytest.mark.parametrize("cpu_workers,policy,dl,prefetch", [(0, "pats", True, True), (0, "fcfs", False, False),
                                                            (3, "pats", True, True), (3, "fcfs", True, False)])
def test_gpu_batches(lib, rc, tiles, expected, batch, depth, cpu_workers, policy, dl, prefetch):
    """The GPU manager running up to 4 or 8 ready h-dome or fill-holes instances
    in one recon_batch launch (tiles of different shapes together), alone or
    beside CPU workers: every tile equals the oracle's chain and every
    instance runs once."""
    gpu_ms = {"hdome": 0.2, "fill_holes": 0.2, "area_threshold": 0.1, "markers": 0.1, "label": 0.05}
    cfg = lib.pipe_config(policy=policy, cpu_workers=cpu_workers, use_gpu=True, window=6, data_locality=dl,
                          conn=8, h=H, area_min=LO, area_max=HI, speedup=SPEEDUP, gpu_ms=gpu_ms,
                          cpu_guard=cpu_workers > 0, prefetch=prefetch, gpu_inflight=depth, gpu_batch=batch)
    outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg, trace=True)
    check(outs, expected[8])
    assert [a + b for a, b in zip(st["ops_cpu"], st["ops_gpu"])] == [len(tiles)] * 5
    seen = sorted((t, op) for t, op, _, _, _ in st["trace"])
    assert seen == sorted((t, op) for t in range(len(tiles)) for op in lib.PIPE_OPS)
    if cpu_workers == 0:
        # with the GPU alone the first h-domes of the window go in one launch:
        # the second is taken before the first is done
        first = [e for e in st["trace"] if e[1] == "hdome"][:2]
        assert len(first) == 2 and first[1][3] < first[0][4], first


def test_gpu_batches_full_size_and_conn4(lib, rc, oracle_mod):
    """Six 4096 x 4096 nuclei-like tiles, 4-connectivity and another dome
    height, in batches of up to 8 with two launches in flight, against the
    oracle's chain."""
    tiles = [synth.config2_tile(seed=synth.seed_for(6, 980 + i))[1] for i in range(6)]
    cfg = lib.pipe_config(policy="pats", cpu_workers=0, use_gpu=True, window=6, conn=4, h=35, area_min=LO,
                          area_max=HI, speedup=SPEEDUP, prefetch=True, io_threads=4, gpu_inflight=2, gpu_batch=8)
    outs, st = lib.recon_pipeline_run(rc.ctx, tiles, cfg)
    for img, o in zip(tiles, outs):
        a = oracle_mod.area_threshold(oracle_mod.fill_holes(oracle_mod.hdome(img, 35, 4), 4), LO, HI, 4)
        lab, n = oracle_mod.label(a, 4)
        assert np.array_equal(o["objects"], a) and np.array_equal(o["markers"], oracle_mod.pre_watershed(a, 4))
        assert np.array_equal(o["labels"], lab) and o["count"] == n
    assert st["ops_gpu"] == [6] * 5
