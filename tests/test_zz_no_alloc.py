"""recon_dilate_noalloc, the entry point that allocates nothing, against
recon_dilate (the same reconstruction with the context's workspace) and the
oracle, through the C ABI.

Two calls in a row on the one fixed device workspace, the second with a
smaller image (so stale ring slots, state words and counters of the first call
are still there when the second starts), then an image above the workspace's
limit, which must be refused before anything is enqueued.  Integer work: the
bar is bit-exact.
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


def _dev(torch_mod, a):
    return torch_mod.from_numpy(np.ascontiguousarray(a)).cuda()


def _assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError("%s: %d pixels differ, first at (%d, %d): got %d want %d"
                             % (what, len(bad), y, x, got[y, x], want[y, x]))


def _case(h, w, seed):
    mask = synth.gaussian_tile(h, w, max(4, round(40 * h * w / 512 ** 2)), seed=seed)
    marker = np.maximum(mask.astype(np.int16) - 30, 0).astype(np.uint8)
    return marker, mask


@pytest.mark.parametrize("conn", [8, 4])
def test_noalloc_matches_dilate_twice_shrinking(torch_mod, lib, oracle_mod, conn):
    # first a 1000 x 1300 tile (4 x 6 blocks of 256 columns, ragged in both
    # directions), then a smaller 300 x 500 one on the same fixed workspace
    cases = [_case(1000, 1300, 71 + conn), _case(300, 500, 91 + conn)]
    with lib.Recon(0) as ctx:
        for k, (marker, mask) in enumerate(cases):
            print("no-alloc call %d: %dx%d conn %d" % (k, mask.shape[0], mask.shape[1], conn), flush=True)
            want = oracle_mod.recon_dilate(marker, mask, conn)
            a = _dev(torch_mod, marker)
            b = _dev(torch_mod, marker)
            km = _dev(torch_mod, mask)
            ctx.dilate_noalloc(a, km, conn)
            st = ctx.last_stats()   # waits with a deadline; raises if the launch was stopped
            assert st["aborted"] == 0
            assert st["dense_visits"] >= 1
            ctx.dilate(b, km, conn)
            ctx.last_stats()
            ga, gb = a.cpu().numpy(), b.cpu().numpy()
            _assert_same(ga, gb, "noalloc vs recon_dilate, call %d" % k)
            _assert_same(ga, want, "noalloc vs oracle, call %d" % k)


def test_noalloc_back_to_back_on_one_stream(torch_mod, lib, oracle_mod):
    # two calls enqueued without a synchronisation between them: the second
    # (smaller) resets the workspace only after the first has finished on the stream
    big, small = _case(700, 900, 5), _case(129, 257, 6)
    with lib.Recon(0) as ctx:
        outs = []
        for marker, mask in (big, small):
            a = _dev(torch_mod, marker)
            km = _dev(torch_mod, mask)
            ctx.dilate_noalloc(a, km, 8)
            outs.append((a, km))
        ctx.last_stats()
        for (a, _), (marker, mask) in zip(outs, (big, small)):
            _assert_same(a.cpu().numpy(), oracle_mod.recon_dilate(marker, mask, 8), "back to back")


def test_noalloc_refuses_images_above_the_limit(torch_mod, lib):
    # 8193 blocks of 32 x 256 pixels: one row of blocks more than the workspace holds
    with lib.Recon(0, block_rows=32) as ctx:
        marker = torch_mod.zeros((32 * 8193, 256), dtype=torch_mod.uint8, device="cuda")
        mask = torch_mod.zeros_like(marker)
        with pytest.raises(lib.ReconError) as e:
            ctx.dilate_noalloc(marker, mask, 8)
        assert e.value.code == lib.RECON_EINVAL
        assert "fixed workspace" in str(e.value)
        # the largest image it takes still runs: 8192 blocks (every one of them
        # queued at the start), here with the marker at the mask, so that the
        # result is the mask itself (rho_I(I) = I)
        g = torch_mod.Generator().manual_seed(11)
        mask = torch_mod.randint(0, 256, (32 * 8192, 256), generator=g, dtype=torch_mod.uint8).cuda()
        marker = mask.clone()
        ctx.dilate_noalloc(marker, mask, 4)
        st = ctx.last_stats()
        assert st["dense_visits"] == 8192
        assert bool((marker == mask).all())
