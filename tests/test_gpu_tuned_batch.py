"""The uneven batch with per-task tuning inside one launch, against the oracle.

The autotuner's choices travel per task (scan rounds, LDS queue capacity and
block rows; the context's queue capacity is the launch's); they change speed,
never bytes.  One graph launch holds tiles of every size bucket and both
connectivities with mixed per-task knobs, and one batch call holds tasks of
all three block heights (one launch per height, side by side); every tile is
compared with the oracle (integer work: bit-exact)."""
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


def _run(torch_mod, ctx, tasks, knobs):
    outs, spec = [], []
    for t, (sr, qc) in zip(tasks, knobs):
        m = torch_mod.from_numpy(t["marker"]).cuda()
        k = torch_mod.from_numpy(t["mask"]).cuda()
        outs.append(m)
        spec.append({"op": "dilate", "image": m, "mask": k, "conn": t["conn"], "scan_rounds": sr,
                     "queue_capacity": qc})
    ctx.batch(spec)
    st = ctx.last_stats()
    return [o.cpu().numpy() for o in outs], st


@pytest.mark.parametrize("block_rows", [64, 32, 16])
def test_mixed_per_task_knobs_in_one_launch(torch_mod, lib, oracle_mod, block_rows):
    tasks = synth.config4_batch(n_tiles=24, scale=0.5)   # sides 256 .. 2048, both connectivities
    rounds = [1, 2, 3, 4, -1]
    qcaps = [64, 256, 512, 1024, 2048]
    knobs = [(rounds[i % len(rounds)], qcaps[(i // 2) % len(qcaps)]) for i in range(len(tasks))]
    with lib.Recon(0, block_rows=block_rows, queue_capacity=2048) as ctx:
        outs, st = _run(torch_mod, ctx, tasks, knobs)
        assert st["aborted"] == 0
        for i, (t, got) in enumerate(zip(tasks, outs)):
            want = oracle_mod.run_task(t)
            assert np.array_equal(got, want), "tile %d (%dx%d, conn %d, knobs %s)" % (
                i, got.shape[0], got.shape[1], t["conn"], knobs[i])


def test_tuned_batch_from_the_cache(torch_mod, lib, oracle_mod):
    """The tuner's choices for this batch (from the committed cache when it was
    measured on these kernels, else the defaults) give the oracle's bytes."""
    from paper_1209_3332_amd import tune
    tasks = synth.config4_batch(n_tiles=16, scale=0.5)
    cache = tune.load_cache()
    devs = [{"op": "dilate", "image": torch_mod.from_numpy(t["marker"]).cuda(),
             "mask": torch_mod.from_numpy(t["mask"]).cuda(), "conn": t["conn"]} for t in tasks]
    bh, qcap, tuned = tune.tuned_batch(cache, devs)
    with lib.Recon(0, block_rows=bh, queue_capacity=qcap) as ctx:
        ctx.batch(tuned)
        ctx.last_stats()
        for i, (t, d) in enumerate(zip(tasks, devs)):
            assert np.array_equal(d["image"].cpu().numpy(), oracle_mod.run_task(t)), "tile %d" % i


@pytest.mark.parametrize("n_tiles", [9, 30])   # direct launches and graph replays per group
def test_mixed_block_heights_in_one_batch(torch_mod, lib, oracle_mod, n_tiles):
    """Per-task block rows of 16, 32 and 64 (and 0, the context's) in one
    recon_batch call, with mixed ops, against the oracle; the statistics sum
    the groups' counters (every block of every task visited at least once)."""
    tasks = synth.config4_batch(n_tiles=n_tiles, scale=0.5)
    heights = [16, 32, 64, 0]
    with lib.Recon(0, block_rows=32, queue_capacity=2048, timing=1) as ctx:
        for rep in range(2):   # twice in a row: the groups' contexts and graphs are reused
            spec, outs, wants, blocks = [], [], [], 0
            for i, t in enumerate(tasks):
                bh = heights[(i + rep) % len(heights)]
                m = torch_mod.from_numpy(t["marker"]).cuda()
                k = torch_mod.from_numpy(t["mask"]).cuda()
                if i % 3 == 2:   # an h-dome of the mask instead
                    spec.append({"op": "hdome", "image": k, "conn": t["conn"], "h": 25, "block_rows": bh})
                    outs.append(k)
                    wants.append(oracle_mod.hdome(t["mask"], 25, t["conn"]))
                else:
                    spec.append({"op": "dilate", "image": m, "mask": k, "conn": t["conn"], "block_rows": bh})
                    outs.append(m)
                    wants.append(oracle_mod.run_task(t))
                rows = bh or 32
                blocks += -(-t["mask"].shape[0] // rows) * -(-t["mask"].shape[1] // 256)
            ctx.batch(spec)
            st = ctx.last_stats()
            assert st["aborted"] == 0 and st["total_ms"] > 0
            assert st["dense_visits"] + st["component_tasks"] > 0
            assert st["dense_visits"] <= blocks
            for i, (o, w) in enumerate(zip(outs, wants)):
                assert np.array_equal(o.cpu().numpy(), w), "tile %d (block rows %s)" % (i, spec[i]["block_rows"])


def test_bad_task_block_rows_is_rejected(torch_mod, lib):
    m = torch_mod.zeros((8, 8), dtype=torch_mod.uint8, device="cuda")
    k = torch_mod.zeros((8, 8), dtype=torch_mod.uint8, device="cuda")
    with lib.Recon(0) as ctx:
        with pytest.raises(lib.ReconError) as e:
            ctx.batch([{"op": "dilate", "image": m, "mask": k, "conn": 8, "block_rows": 48}])
        assert e.value.code == lib.RECON_EINVAL
