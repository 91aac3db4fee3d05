"""The uneven batch with per-task tuning inside one launch, against the oracle.

The autotuner's choices travel per task (scan rounds, LDS queue capacity) and
per launch (block rows, the context's queue capacity); they change speed,
never bytes.  One graph launch holds tiles of every size bucket and both
connectivities with mixed per-task knobs, and every tile is compared with the
oracle (integer work: bit-exact)."""
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
