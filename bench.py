#!/usr/bin/env python3
"""Benchmark of the reconstruction path on one MI355X.

Workload (the configuration the headline metric is quoted on): a batch of 64
uint8 4096 x 4096 tiles, 8-connectivity -- 56 nuclei-like tiles (the 512 x 512
generator scaled to area: 2560 Gaussians, sigma U[4,12], amplitude U[40,200],
noise [-8,8]; marker max(I - 30, 0)) and 8 adversarial spiral-corridor tiles
(1-pixel corridor, one chain of 8.39 M pixels, a single seed at one end).

A step is one batched launch sequence (recon_batch: one HIP-graph replay of
reset -> dense pass -> border seeding -> revisit drain) over the whole batch,
with every input already resident in device memory; each step reconstructs its
own untouched copy of the markers, so nothing is skipped or cached.  Printed as
one JSON line: batched Mpixel/s (value), the same 64 tiles as 64 plain per-tile
calls, per-tile latency percentiles, per-kernel durations measured with HIP
events inside the timed steps, the dense kernel's roofline, and the CPU oracle
timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "recon Mpixel/s, 4K² uint8 8-conn, batched vs per-tile; p99 latency; %HBM"
HBM_PEAK_GBS = 8000.0
BYTES_PER_PX = 3.0   # algorithmic: read mask, read marker, write result


def _gen_tile(args):
    import synth
    i, size = args
    mask = synth.scaled_config1_tile(size, size, synth.seed_for(3, i))
    return i, synth.hdome_marker(mask, 30), mask


def make_batch(n_tiles, size, workers):
    """Host arrays of the batch: (kind, marker, mask) per tile."""
    import multiprocessing as mp
    import synth
    nuclei = [i for i in range(n_tiles) if i % 8 != 7]
    out = [None] * n_tiles
    with mp.get_context("fork").Pool(workers) as pool:
        for i, marker, mask in pool.imap_unordered(_gen_tile, [(i, size) for i in nuclei]):
            out[i] = ("nuclei", marker, mask)
    spirals = {}
    for i in range(n_tiles):
        if i % 8 == 7:
            where = "outer" if i % 16 == 7 else "inner"
            if where not in spirals:
                spirals[where] = synth.spiral_tile(size, size, where)[:2]
            out[i] = ("spiral", spirals[where][0], spirals[where][1])
    return out


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(batch, budget_s=20.0):
    """The oracle, as it is, on the host cores: a bag of tiles over a thread pool."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    cores = len(os.sched_getaffinity(0))
    nuclei = [b for b in batch if b[0] == "nuclei"]
    # one tile single-threaded to size the sample to about budget_s of CPU work
    t = time.perf_counter()
    oracle.recon_dilate(nuclei[0][1], nuclei[0][2], 8)
    per_tile = time.perf_counter() - t
    n = max(1, min(len(nuclei), int(budget_s / max(per_tile, 1e-3))))
    sample = nuclei[:n]
    t = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(lambda b: oracle.recon_dilate(b[1], b[2], 8), sample))
    wall = time.perf_counter() - t
    px = sum(b[2].size for b in sample)
    return {"value": px / wall / 1e6, "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
            "sample": "%d nuclei tiles of %dx%d (8-conn), one tile per thread; single-core %.1f Mpixel/s"
                      % (n, nuclei[0][2].shape[0], nuclei[0][2].shape[1], nuclei[0][2].size / per_tile / 1e6)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tiles", type=int, default=64)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--block-rows", type=int, default=0)
    ap.add_argument("--scan-rounds", type=int, default=0)
    ap.add_argument("--queue", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-tile", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the reconstruction shards by tile with no "
              "communication, and this build measures the single-GPU path only (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import oracle
    import paper_1209_3332_amd as recon

    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    batch = make_batch(args.tiles, args.size, args.workers)
    log("generated %d tiles in %.1f s" % (len(batch), time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    masks = [torch.from_numpy(b[2]).to(dev) for b in batch]
    pristine = [torch.from_numpy(b[1]).to(dev) for b in batch]
    n_sets = args.warmup + args.steps
    sets = [[p.clone() for p in pristine] for _ in range(n_sets)]
    torch.cuda.synchronize()
    px_total = sum(m.numel() for m in masks)

    cfg = dict(timing=1)
    if args.block_rows:
        cfg["block_rows"] = args.block_rows
    if args.scan_rounds:
        cfg["scan_rounds"] = args.scan_rounds
    if args.queue:
        cfg["queue_capacity"] = args.queue
    ctx = recon.Recon(0, **cfg)
    stream = torch.cuda.current_stream()

    def tasks_of(markers):
        return [{"op": "dilate", "image": markers[i], "mask": masks[i], "conn": 8} for i in range(len(masks))]

    # ---- batched: warmup, then exactly `steps` timed steps
    for s in range(args.warmup):
        ctx.batch(tasks_of(sets[s]), stream)
        ctx.last_stats()
    torch.cuda.synchronize()
    kstats = []
    t_start = time.perf_counter()
    for s in range(args.warmup, n_sets):
        ctx.batch(tasks_of(sets[s]), stream)
        kstats.append(ctx.last_stats())   # waits for the step; per-kernel HIP event times
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps
    value = px_total / (wall / args.steps) / 1e6
    log("batched: %.2f ms/step, %.0f Mpixel/s" % (ms_per_step, value))

    # ---- parity on the last step: spirals must equal their mask; one nuclei tile against the oracle
    last = sets[-1]
    parity = {"checked": [], "ok": True}
    for i, b in enumerate(batch):
        if b[0] == "spiral":
            ok = bool(torch.equal(last[i], masks[i]))
            parity["checked"].append("spiral %d" % i)
            parity["ok"] &= ok
    want = oracle.recon_dilate(batch[0][1], batch[0][2], 8)
    parity["ok"] &= bool(np.array_equal(last[0].cpu().numpy(), want))
    parity["checked"].append("nuclei 0 vs oracle")

    # ---- per-tile: the same tiles as plain calls
    per_tile = None
    if not args.no_per_tile:
        work = [p.clone() for p in pristine]
        torch.cuda.synchronize()
        lat = []
        t = time.perf_counter()
        for i in range(len(masks)):
            ctx.dilate(work[i], masks[i], 8, stream)
            lat.append(ctx.last_stats()["total_ms"])
        torch.cuda.synchronize()
        wall_pt = time.perf_counter() - t
        nuc = [lat[i] for i, b in enumerate(batch) if b[0] == "nuclei"]
        spi = [lat[i] for i, b in enumerate(batch) if b[0] == "spiral"]
        per_tile = {"value": px_total / wall_pt / 1e6, "unit": "Mpixel/s", "ms_total": wall_pt * 1e3,
                    "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                                   "nuclei_p50": percentile(nuc, 50), "nuclei_p99": percentile(nuc, 99),
                                   "spiral_p50": percentile(spi, 50), "spiral_max": max(spi) if spi else None}}
        log("per-tile: %.0f Mpixel/s, p50 %.2f ms, p99 %.2f ms" % (per_tile["value"], per_tile["latency_ms"]["p50"],
                                                                   per_tile["latency_ms"]["p99"]))

    # ---- per-kernel durations (HIP events on the launch stream, averaged over the timed steps)
    avg = lambda k: sum(s[k] for s in kstats) / len(kstats)
    kernels = {"dense_pass_ms": avg("dense_ms"), "border_seed_ms": avg("seed_ms"),
               "revisit_drain_ms": avg("drain_ms"), "launch_ms": avg("total_ms"),
               "revisits": avg("revisits"), "queue_overflows": avg("queue_overflows")}
    dense_gbs = BYTES_PER_PX * px_total / (kernels["dense_pass_ms"] * 1e-3) / 1e9
    roofline = {"kernel": "dense_pass", "bound": "hbm", "achieved": dense_gbs, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dense_gbs / HBM_PEAK_GBS, "traffic": None,
                "bytes_per_px": BYTES_PER_PX,
                "whole_launch_GBs": BYTES_PER_PX * px_total / (kernels["launch_ms"] * 1e-3) / 1e9}

    out = {"metric": METRIC, "value": value, "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "batch of %d uint8 %dx%d tiles, 8-conn: %d nuclei-like (h=30) + %d spiral corridors"
                                  % (args.tiles, args.size, args.size,
                                     sum(b[0] == "nuclei" for b in batch), sum(b[0] == "spiral" for b in batch)),
                      "tiles": args.tiles, "tile": [args.size, args.size], "conn": 8, "mode": "batched hipGraph",
                      "block_rows": ctx.cfg.get("block_rows", 32)},
           "per_tile": per_tile, "kernels": kernels, "roofline": roofline, "parity": parity}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(batch)
        log("cpu baseline: %.1f Mpixel/s on %d cores" % (out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"]))
    ctx.close()
    print(json.dumps(out), flush=True)
    if not parity["ok"]:
        sys.exit(1)


if __name__ == "__main__":
    main()
