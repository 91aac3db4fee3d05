"""Autotuner bookkeeping (CPU only): size buckets, defaults, per-task knobs."""
import numpy as np

from paper_1209_3332_amd import tune


def test_buckets():
    assert tune.bucket_of(512, 512) == "small"
    assert tune.bucket_of(1024, 1024) == "small"
    assert tune.bucket_of(2048, 2048) == "medium"
    assert tune.bucket_of(4096, 4096) == "large"


def test_defaults_without_cache():
    cfg = tune.config_for({}, 4096, 4096, 8)
    assert cfg["block_rows"] in tune.BLOCK_ROWS and cfg["queue_capacity"] in tune.QUEUE_CAPACITY


def test_tuned_batch_picks_per_bucket():
    cache = {"arch": "gfx950", "gfx950": {
        "small/conn8": {"block_rows": 16, "scan_rounds": 1, "queue_capacity": 512},
        "large/conn4": {"block_rows": 64, "scan_rounds": 4, "queue_capacity": 8192}}}
    tasks = [{"op": "dilate", "image": np.zeros((512, 512), np.uint8), "mask": None, "conn": 8},
             {"op": "dilate", "image": np.zeros((4096, 4096), np.uint8), "mask": None, "conn": 4}]
    bh, qmax, out = tune.tuned_batch(cache, tasks)
    assert bh == 64                      # the bucket holding most pixels
    assert qmax == 8192                  # the context sizes LDS for the largest queue
    assert (out[0]["scan_rounds"], out[0]["queue_capacity"], out[0]["block_rows"]) == (1, 512, 16)
    assert (out[1]["scan_rounds"], out[1]["queue_capacity"], out[1]["block_rows"]) == (4, 8192, 64)


def test_cache_is_stamped_and_stale_caches_are_ignored(tmp_path):
    import json
    good = {"arch": "gfx950", "gfx950": {}, "kernel_sha": tune.kernel_sha(), "hip_runtime": "x"}
    stale = dict(good, kernel_sha="0000000000000000")
    assert tune.cache_valid(good) and tune.cache_valid(good, "x") and not tune.cache_valid(good, "y")
    assert not tune.cache_valid(stale) and not tune.cache_valid({})
    p = tmp_path / "c.json"
    p.write_text(json.dumps(stale))
    assert tune.load_cache(str(p), check_runtime=False) == {}
    p.write_text(json.dumps(good))
    assert tune.load_cache(str(p), check_runtime=False) == good
