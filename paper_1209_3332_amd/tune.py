"""Autotuner for librecon: block rows, LDS queue capacity and scan-pass rounds.

The knobs change speed, never bytes (the reconstruction is unique).  All three
travel per task, so one batched call can use a different setting for each size
bucket: scan rounds and queue capacity inside one launch, block rows (which set
the kernels' LDS layout) by running each block height's tasks as a launch of
their own, side by side with the others.

    python -m paper_1209_3332_amd.tune [--out FILE] [--reps N]

measures every combination on synthetic nuclei-like tiles of each size bucket
and connectivity (timed with HIP events around the launch) and writes a JSON
cache keyed by the GPU's architecture, stamped with a hash of the kernel
source and the HIP runtime version it was measured on: a cache taken on other
kernels or another runtime is ignored (defaults apply) until the tuner runs
again.  `tuned_batch()` applies a cache to a list of tasks.
"""
from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.environ.get("RECON_TUNE_CACHE", os.path.join(HERE, "tune_cache.json"))

BLOCK_ROWS = (16, 32, 64)
QUEUE_CAPACITY = (512, 2048, 8192)
SCAN_ROUNDS = (-1, 1, 2, 3, 4)   # -1: no sweep on first visits (seed and queue only)
# size buckets by tile area (pixels): representative side length of each
BUCKETS = (("small", 1 << 20, 768), ("medium", 6 << 20, 2048), ("large", 1 << 62, 4096))


KERNEL_SOURCES = ("kernels.hpp", "component.hpp", "label.hpp", "recon.hip")


def kernel_sha() -> str:
    """Hash of the device code the tuning depends on."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def runtime_version() -> str:
    import torch
    return str(getattr(torch.version, "hip", None) or "unknown")


def cache_valid(cache: dict, runtime: str | None = None) -> bool:
    """True if the cache was measured on the current kernels (and, when
    `runtime` is given, on that HIP runtime)."""
    if not cache or cache.get("kernel_sha") != kernel_sha():
        return False
    return runtime is None or cache.get("hip_runtime") == runtime


def bucket_of(h: int, w: int) -> str:
    area = h * w
    for name, limit, _ in BUCKETS:
        if area <= limit:
            return name
    return BUCKETS[-1][0]


def load_cache(path: str = DEFAULT_CACHE, check_runtime: bool = True) -> dict:
    """The tuning cache, or {} when there is none or it was measured on other
    kernel source or another HIP runtime."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        cache = json.load(f)
    return cache if cache_valid(cache, runtime_version() if check_runtime else None) else {}


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def config_for(cache: dict, h: int, w: int, conn: int, arch: str | None = None) -> dict:
    """Tuned {block_rows, scan_rounds, queue_capacity} for a tile (defaults if untuned)."""
    entry = cache.get(arch or cache.get("arch", ""), {}) if cache else {}
    return entry.get("%s/conn%d" % (bucket_of(h, w), conn),
                     {"block_rows": 32, "scan_rounds": 3, "queue_capacity": 2048})


def tuned_batch(cache: dict, tasks: list) -> tuple[int, int, list]:
    """Block rows for the context (the choice of the bucket holding most pixels),
    the context's queue capacity (the largest per-task choice: it sizes the LDS
    of every workgroup) and the tasks with their per-task block rows, scan
    rounds and queue capacity filled in."""
    weight = {}
    out = []
    qmax = 0
    for t in tasks:
        h, w = t["image"].shape
        cfg = config_for(cache, h, w, t.get("conn", 8))
        weight[cfg["block_rows"]] = weight.get(cfg["block_rows"], 0) + h * w
        qmax = max(qmax, cfg["queue_capacity"])
        out.append(dict(t, scan_rounds=cfg["scan_rounds"], queue_capacity=cfg["queue_capacity"],
                        block_rows=cfg["block_rows"]))
    bh = max(weight, key=weight.get) if weight else 32
    return bh, qmax or 2048, out


def _workload(side: int, conn: int, n_px_target: int):
    import synth
    n = max(1, n_px_target // (side * side))
    tiles = []
    for i in range(n):
        mask = synth.scaled_config1_tile(side, side, synth.seed_for(9, 1000 * side + i))
        tiles.append((synth.hdome_marker(mask, 10 + (i * 7) % 31), mask))
    return tiles


def tune(reps: int = 3, n_px_target: int = 48 << 20, log=print) -> dict:
    import torch
    import paper_1209_3332_amd as recon

    dev = torch.device("cuda:0")
    result = {}
    for bucket, _, side in BUCKETS:
        for conn in (4, 8):
            tiles = _workload(side, conn, n_px_target)
            masks = [torch.from_numpy(m).to(dev) for _, m in tiles]
            pristine = [torch.from_numpy(j).to(dev) for j, _ in tiles]
            work = [p.clone() for p in pristine]
            best = None
            for bh, qc in itertools.product(BLOCK_ROWS, QUEUE_CAPACITY):
                # the context's queue capacity sizes every workgroup's LDS (and so
                # the occupancy): tune it together with the per-task value
                with recon.Recon(0, block_rows=bh, queue_capacity=qc, timing=1) as ctx:
                    for sr in SCAN_ROUNDS:
                        times = []
                        for _ in range(reps + 1):
                            for w_, p_ in zip(work, pristine):
                                w_.copy_(p_)
                            ctx.batch([{"op": "dilate", "image": w_, "mask": m_, "conn": conn,
                                        "scan_rounds": sr, "queue_capacity": qc}
                                       for w_, m_ in zip(work, masks)])
                            times.append(ctx.last_stats()["total_ms"])
                        ms = statistics.median(times[1:])
                        if best is None or ms < best[0]:
                            best = (ms, {"block_rows": bh, "scan_rounds": sr, "queue_capacity": qc})
            px = sum(m.numel() for m in masks)
            best[1]["ms"] = best[0]
            best[1]["mpx_s"] = px / best[0] / 1e3
            result["%s/conn%d" % (bucket, conn)] = best[1]
            log("%s conn%d: %s" % (bucket, conn, best[1]))
    return {"arch": _arch(), _arch(): result, "kernel_sha": kernel_sha(), "hip_runtime": runtime_version()}


def main():
    ap = argparse.ArgumentParser(description="tune librecon for this GPU")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    res = tune(args.reps, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
