"""Serving loop (recon_submit / recon_poll / recon_wait) on the GPU.

Each request's result must be the same bytes alone and inside a mix of
concurrent requests (the reconstruction is unique, so the tolerance is 0), and
equal to the oracle; admission must push back (RECON_EAGAIN) instead of
over-committing when the slot or memory cap is reached.
"""
import time

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


def _task(rng, i):
    h, w = int(rng.integers(64, 900)), int(rng.integers(64, 900))
    conn = int(rng.choice([4, 8]))
    mask = synth.scaled_config1_tile(h, w, 9000 + i)
    return {"op": "dilate", "marker": synth.hdome_marker(mask, int(rng.integers(10, 41))), "mask": mask,
            "conn": conn}


def _submit_all(torch_mod, ctx, tasks, lib, timeout_s=60.0):
    # every image is uploaded first (one synchronisation), then the requests go
    # in a burst, so that they arrive while earlier ones are on the GPU
    bufs, tickets = [], []
    for t in tasks:
        bufs.append((torch_mod.from_numpy(t["marker"]).cuda(), torch_mod.from_numpy(t["mask"]).cuda()))
    torch_mod.cuda.synchronize()
    for t, (m, k) in zip(tasks, bufs):
        deadline = time.time() + timeout_s
        while True:
            try:
                tickets.append(ctx.submit("dilate", m, k, t["conn"]))
                break
            except lib.ReconAgain:
                assert time.time() < deadline, "admission never freed up"
                time.sleep(0.001)   # earlier requests complete in the background
    for tk in tickets:
        ctx.wait(tk, int(timeout_s * 1e6))
    return [m.cpu().numpy() for m, _ in bufs]


def test_alone_and_in_the_mix(torch_mod, lib, oracle_mod):
    rng = np.random.default_rng(2024)
    probe = _task(rng, 0)
    want = oracle_mod.run_task(probe)
    with lib.Recon(0) as ctx:
        alone = _submit_all(torch_mod, ctx, [probe], lib)[0]
        assert np.array_equal(alone, want)
        mix = [_task(rng, i) for i in range(1, 30)]
        mix.insert(11, probe)
        outs = _submit_all(torch_mod, ctx, mix, lib)
        assert np.array_equal(outs[11], alone)
        for i, (t, got) in enumerate(zip(mix, outs)):
            assert np.array_equal(got, oracle_mod.run_task(t)), "request %d" % i
        st = ctx.serve_stats()
        # the requests overlapped on the device: some launch held several of them
        # or several lanes ran at once
        assert st["requests"] == 31 and (st["max_batch"] > 1 or st["max_busy_lanes"] > 1), st
        ctx.serve_stop()


def test_tickets_complete_with_their_own_tile(torch_mod, lib, oracle_mod):
    """A launch holding large and small reconstructions completes each ticket
    when its own tile converges: small tiles do not wait for the large ones
    (counted as early completions), and every result equals the oracle."""
    rng = np.random.default_rng(99)
    big = []
    for i in range(3):
        mask = synth.scaled_config1_tile(2048, 2048, 9500 + i)
        big.append({"op": "dilate", "marker": synth.hdome_marker(mask, 20), "mask": mask, "conn": 8})
    small = [_task(rng, 200 + i) for i in range(40)]
    tasks = [big[0], big[1], big[2]] + small
    with lib.Recon(0) as ctx:
        bufs = [(torch_mod.from_numpy(t["marker"]).cuda(), torch_mod.from_numpy(t["mask"]).cuda()) for t in tasks]
        torch_mod.cuda.synchronize()
        tickets = [ctx.submit("dilate", m, k, t["conn"]) for t, (m, k) in zip(tasks, bufs)]
        # each result is copied out the moment its own ticket completes, while
        # the rest of its launch may still run on the device
        got = [None] * len(tasks)
        deadline = time.time() + 60
        while any(g is None for g in got):
            assert time.time() < deadline, "tickets did not complete"
            for i, tk in enumerate(tickets):
                if got[i] is None and ctx.poll(tk):
                    got[i] = bufs[i][0].cpu().numpy()
        st = ctx.serve_stats()
        for i, t in enumerate(tasks):
            assert np.array_equal(got[i], oracle_mod.run_task(t)), "request %d" % i
        assert st["max_batch"] > 1, st
        assert st["early_completions"] > 0, st
        ctx.serve_stop()


def test_admission_backpressure(torch_mod, lib, oracle_mod):
    rng = np.random.default_rng(7)
    # a long-running request first (a spiral corridor: one long propagation chain)
    # keeps its slot busy while the quick ones are submitted back to back
    s_marker, s_mask, _ = synth.spiral_tile(1024, 1024, "outer")
    tasks = [{"op": "dilate", "marker": s_marker, "mask": s_mask, "conn": 8}]
    tasks += [_task(rng, 100 + i) for i in range(12)]
    with lib.Recon(0, serve_slots=3) as ctx:
        bufs = [(torch_mod.from_numpy(t["marker"]).cuda(), torch_mod.from_numpy(t["mask"]).cuda()) for t in tasks]
        torch_mod.cuda.synchronize()
        tickets, again = [], 0
        for t, (m, k) in zip(tasks, bufs):
            while True:
                try:
                    tickets.append(ctx.submit("dilate", m, k, t["conn"]))
                    break
                except lib.ReconAgain:
                    again += 1
                    # wait for the oldest outstanding ticket, then try again
                    pending = [tk for tk in tickets if tk is not None]
                    ctx.wait(pending[0], 60_000_000)
                    tickets[tickets.index(pending[0])] = None
        for tk in tickets:
            if tk is not None:
                ctx.wait(tk, 60_000_000)
        assert again > 0   # the slot cap of 3 was hit
        for t, (m, _) in zip(tasks, bufs):
            assert np.array_equal(m.cpu().numpy(), oracle_mod.run_task(t))
        # stop, then serving restarts on the next submit
        ctx.serve_stop()
        t = tasks[1]
        m = torch_mod.from_numpy(t["marker"]).cuda()
        k = torch_mod.from_numpy(t["mask"]).cuda()
        torch_mod.cuda.synchronize()
        tk = ctx.submit("dilate", m, k, t["conn"])
        assert not isinstance(tk, bool)
        ctx.wait(tk, 60_000_000)
        assert np.array_equal(m.cpu().numpy(), oracle_mod.run_task(t))


def test_unknown_ticket(torch_mod, lib):
    with lib.Recon(0) as ctx:
        with pytest.raises(lib.ReconError):
            ctx.poll(12345)


def test_abandoned_launch_fails_its_requests(torch_mod, lib):
    """A serving launch that its scheduler gives up (the context's test hook
    makes every block claim fail, so the launch aborts at once) fails the
    requests it had not completed: recon_wait reports RECON_EDEVICE instead of
    handing out an unfinished reconstruction."""
    mask = synth.gaussian_tile(100, 300, 5, seed=3)
    with lib.Recon(0, test_fault=1) as ctx:
        m = torch_mod.from_numpy(synth.hdome_marker(mask, 30)).cuda()
        k = torch_mod.from_numpy(mask).cuda()
        torch_mod.cuda.synchronize()
        tk = ctx.submit("dilate", m, k, 8)
        with pytest.raises(lib.ReconError) as e:
            ctx.wait(tk, 30_000_000)
        assert e.value.code == lib.RECON_EDEVICE
