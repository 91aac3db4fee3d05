#!/usr/bin/env python3
"""Benchmark of the reconstruction path on one MI355X.

Headline workload (the 4K-tile configuration the metric is quoted on): one
uint8 4096 x 4096 nuclei-like tile (~3000 Gaussians, sigma U[3,8], amplitude
U[60,220], background 30, noise [-10,10]).  A step is the tile's whole hot
path: reconstruction by dilation with 8-connectivity from the marker
max(I - 20, 0) and fill-holes (8-connected background) of its binary copy
255 * (I > 120), both in one batched launch (--step-mode plain: two plain
per-tile calls; the plain form is also timed as a section of its own).  Every
step works on its own untouched copies of the inputs, all resident in device
memory before the timed region; `value` = pixels processed (2 x 16.78 M per
step) / time.

Alongside, in the same run: the per-kernel HIP-event durations of the timed
steps and the dominant kernel's roofline (with the HBM traffic of the
committed counter summary when it was taken on the current kernel source);
erosion, h-dome and regional maxima; labelling and the area filter; the
distance transform and Pre-Watershed markers; a 64-tile batch of 4096 x 4096
tiles (every eighth a 4096 x 4096 spiral corridor, which takes the component
route) and an uneven 256-tile autotuned batch against per-tile calls; the
serving loop at arrival rates from 50 to 2000 tiles/s; the co-scheduled tile
pipeline (h-dome, fill-holes, area filter, markers, labels of host tiles on the
GPU and the host cores, FCFS against PATS, with and without data locality).
Last comes the oracle leg: the CPU
oracle timed on the host cores on a bounded sample, then the comparison of
every section's recorded outputs with the oracle (the only part of this
script that runs the oracle; --no-cpu-baseline skips it).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "recon Mpixel/s, 4K² uint8 8-conn, batched vs per-tile; p99 latency; %HBM"
HBM_PEAK_GBS = 8000.0
BYTES_DILATE = 3.0   # algorithmic bytes per pixel: read mask, read marker, write result
BYTES_FILL = 2.0     # read image, write result (the marker is implicit)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(x for x in xs if x is not None)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


KERNEL_SOURCES = [os.path.join(ROOT, "paper_1209_3332_amd", "csrc", f)
                  for f in ("kernels.hpp", "component.hpp", "label.hpp", "recon.hip")]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "revisit_drain_hbm_traffic.md")


def kernel_sha():
    """Hash of the device code and its launch configuration (the library's sources)."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None if
    there is none or it was taken on other kernel source."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"^TRAFFIC_JSON (\{.*\})$", text, re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_sha") != kernel_sha() or kernel not in d.get("bytes_per_launch", {}):
        return None
    return d["bytes_per_launch"][kernel]


def _gen_tile(args):
    import synth
    i, size = args
    mask = synth.scaled_config1_tile(size, size, synth.seed_for(3, i))
    return i, synth.hdome_marker(mask, 30), mask


def make_batch(n_tiles, size, workers, spiral_size):
    """Host arrays of the batch: (kind, marker, mask) per tile; tiles i = 7 (mod 8) are spirals."""
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
                spirals[where] = synth.spiral_tile(spiral_size, spiral_size, where)[:2]
            out[i] = ("spiral", spirals[where][0], spirals[where][1])
    return out


# Comparisons with the oracle are deferred: the sections record host copies of
# their GPU outputs with the oracle call that must reproduce them, and the
# cpu_baseline leg -- the only part of this script that runs the oracle --
# evaluates them after every GPU section has finished (with --no-cpu-baseline
# the parity fields stay null).
CHECKS = []


def defer_check(path, got, fn, *args, rate_path=None, px=None):
    """path: keys into the output line where the verdict goes; got: host array
    (or (labels, count) for the labelling); fn: name of the oracle function;
    rate_path: where the oracle's single-core Mpixel/s on px pixels goes."""
    CHECKS.append({"path": path, "got": got, "fn": fn, "args": args, "rate_path": rate_path, "px": px})


def _set_at(out, path, value):
    node = out
    for key in path[:-1]:
        node = node[key]
    node[path[-1]] = value


def run_checks(out, workers=4):
    """The oracle leg: evaluate every deferred comparison (on a thread pool: the
    oracle runs in C without the interpreter lock); returns True if all agree.
    A path checked several times holds the conjunction of its verdicts."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle

    def solve(c):
        t0 = time.perf_counter()
        if c["fn"] == "pipeline_chain":
            # the tile pipeline's outputs: hdome -> fill-holes -> area filter,
            # then the markers and the labels of the filtered image
            img, h, conn, lo, hi = c["args"]
            a = oracle.area_threshold(oracle.fill_holes(oracle.hdome(img, h, conn), conn), lo, hi, conn)
            want = (a, oracle.pre_watershed(a, conn), oracle.label(a, conn))
        else:
            want = getattr(oracle, c["fn"])(*c["args"])
        return want, time.perf_counter() - t0

    # the comparisons that report a single-core rate run alone, the others in parallel
    timed = [c for c in CHECKS if c["rate_path"]]
    rest = [c for c in CHECKS if not c["rate_path"]]
    results = {id(c): solve(c) for c in timed}
    with ThreadPoolExecutor(max(1, workers)) as ex:
        for c, r in zip(rest, ex.map(solve, rest)):
            results[id(c)] = r
    all_ok = True
    for c in CHECKS:
        want, dt = results[id(c)]
        if c["fn"] == "label":
            ok = bool(np.array_equal(c["got"][0], want[0]) and c["got"][1] == want[1])
        elif c["fn"] == "pipeline_chain":
            g = c["got"]
            ok = bool(np.array_equal(g["objects"], want[0]) and np.array_equal(g["markers"], want[1])
                      and np.array_equal(g["labels"], want[2][0]) and g["count"] == want[2][1])
        else:
            ok = bool(np.array_equal(c["got"], want))
        if c["path"][-1] == "mismatches":     # sampled serving results: count the bad ones
            node = out
            for key in c["path"][:-1]:
                node = node[key]
            node["checked"] = node.get("checked", 0) + 1
            node["mismatches"] = node.get("mismatches", 0) + int(not ok)
        else:
            node = out
            for key in c["path"][:-1]:
                node = node[key]
            prev = node.get(c["path"][-1])
            node[c["path"][-1]] = ok if prev is None else bool(prev and ok)
        if c["rate_path"]:
            _set_at(out, c["rate_path"], c["px"] / dt / 1e6)
        all_ok &= ok
    return all_ok


def cpu_baseline(marker, mask, binary, budget_s=20.0):
    """The oracle, as it is, on the host cores: copies of the headline step over a thread pool."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    cores = len(os.sched_getaffinity(0))
    t = time.perf_counter()
    oracle.recon_dilate(marker, mask, 8)
    oracle.fill_holes(binary, 8)
    one = time.perf_counter() - t
    n = max(1, int(budget_s / max(one, 1e-3)))
    t = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(lambda _: (oracle.recon_dilate(marker, mask, 8), oracle.fill_holes(binary, 8)), range(n)))
    wall = time.perf_counter() - t
    px = 2 * mask.size * n
    return {"value": px / wall / 1e6, "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
            "sample": "%d copies of the headline step (dilate + fill-holes of one %dx%d tile), one per thread; "
                      "single-core %.2f Mpixel/s" % (n, mask.shape[0], mask.shape[1], 2 * mask.size / one / 1e6)}


def headline(recon, torch, cfg, marker, mask, binary, steps, warmup, mode):
    """The headline step on one tile -- 8-conn reconstruction by dilation of
    (max(I - 20, 0), I) and 8-conn fill-holes of 255 * (I > 120) -- timed over
    `steps` steps after `warmup`, each step on its own untouched inputs resident
    in HBM.  mode "batched": both operations in one recon_batch launch per
    step; "plain": recon_dilate then recon_fill_holes.  Returns throughput,
    the kernels' durations from the library's events on the launch stream, the
    parity of the last step, and the roofline of the dominant kernel."""
    import numpy as np
    dev = torch.device("cuda:0")
    d_mask = torch.from_numpy(mask).to(dev)
    n_sets = warmup + steps
    markers = [torch.from_numpy(marker).to(dev) for _ in range(n_sets)]
    images = [torch.from_numpy(binary).to(dev) for _ in range(n_sets)]
    torch.cuda.synchronize()
    ctx = recon.Recon(0, **cfg)
    stream = torch.cuda.current_stream()

    def step(s):
        if mode == "batched":
            ctx.batch([{"op": "dilate", "image": markers[s], "mask": d_mask, "conn": 8},
                       {"op": "fill_holes", "image": images[s], "conn": 8}], stream)
        else:
            ctx.dilate(markers[s], d_mask, 8, stream)
            ctx.fill_holes(images[s], 8, stream)

    for s in range(warmup):
        step(s)
    torch.cuda.synchronize()
    # the timed region: launches back to back, one synchronisation at the end
    t_start = time.perf_counter()
    for s in range(warmup, n_sets):
        step(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / steps
    value = 2 * mask.size / (wall / steps) / 1e6
    log("headline (%s): %.3f ms/step, %.0f Mpixel/s" % (mode, ms_per_step, value))
    # kernel durations of every timed launch, from the library's HIP events on
    # the launch stream (plain: launch 2k is step k's dilate, 2k+1 its fill-holes)
    per_step = 1 if mode == "batched" else 2
    n_q = min(per_step * steps, 64)   # the library keeps the marks of the last 64 launches
    times = [ctx.launch_times(back) for back in range(n_q - 1, -1, -1)]
    groups = {"dilate + fill_holes": times} if mode == "batched" else {"dilate": times[0::2],
                                                                        "fill_holes": times[1::2]}
    # counters of one more (untimed) launch of each kind
    spare_m = torch.from_numpy(marker).to(dev)
    spare_i = torch.from_numpy(binary).to(dev)
    stats = {}
    if mode == "batched":
        ctx.batch([{"op": "dilate", "image": spare_m, "mask": d_mask, "conn": 8},
                   {"op": "fill_holes", "image": spare_i, "conn": 8}], stream)
        stats["dilate + fill_holes"] = ctx.last_stats()
    else:
        ctx.dilate(spare_m, d_mask, 8, stream)
        stats["dilate"] = ctx.last_stats()
        ctx.fill_holes(spare_i, 8, stream)
        stats["fill_holes"] = ctx.last_stats()
    # the last step's outputs, compared with the oracle by the oracle leg
    outputs = {"dilate": markers[-1].cpu().numpy(), "fill_holes": images[-1].cpu().numpy()}
    ctx.close()

    avg = lambda xs, k: sum(x[k] for x in xs) / len(xs)
    kernels = {}
    op_bytes = {"dilate": BYTES_DILATE * mask.size, "fill_holes": BYTES_FILL * mask.size}
    ops_of = {"dilate + fill_holes": ("dilate", "fill_holes"), "dilate": ("dilate",), "fill_holes": ("fill_holes",)}
    for name, ts in groups.items():
        st = stats[name]
        # which operations the launch completed in revisit_drain and which in the
        # component route (the binary fill-holes takes the route; the grey
        # reconstruction the block visits)
        on_route = ("fill_holes",) if st["component_tasks"] == 1 and "fill_holes" in ops_of[name] else ()
        kernels[name] = {"dense_pass_ms": avg(ts, "dense_ms"), "border_seed_ms": avg(ts, "seed_ms"),
                         "revisit_drain_ms": avg(ts, "drain_ms"), "component_route_ms": avg(ts, "route_ms"),
                         "launch_ms": avg(ts, "total_ms"),
                         "dense_visits": st["dense_visits"], "revisits": st["revisits"], "reruns": st["reruns"],
                         "queue_overflows": st["queue_overflows"], "component_tasks": st["component_tasks"],
                         "ops_in_revisit_drain": [o for o in ops_of[name] if o not in on_route],
                         "ops_in_component_route": list(on_route)}
    # dominant kernel (by average duration) and its roofline.  Algorithmic bytes
    # per the method's own traffic: 3 B/px for a reconstruction (read the mask,
    # read the marker, write the result), 2 B/px for a fill-holes (read the
    # image, write the result), counted for the operations that kernel
    # completes.  The bytes a visit schedule moves (3 B/px of a block per
    # visit, first or later) are reported beside them as per_visit_bytes.
    bh = cfg.get("block_rows", 32)
    cand = []
    for name, kv in kernels.items():
        cand.append(("revisit_drain (%s)" % name, kv["revisit_drain_ms"],
                     sum(op_bytes[o] for o in kv["ops_in_revisit_drain"]),
                     3.0 * bh * 256 * (kv["revisits"] + kv["dense_visits"])))
        if kv["ops_in_component_route"]:
            cand.append(("component route (%s)" % name, kv["component_route_ms"],
                         sum(op_bytes[o] for o in kv["ops_in_component_route"]), None))
    dom = max(cand, key=lambda c: c[1])
    achieved = dom[2] / (dom[1] * 1e-3) / 1e9
    traffic = committed_traffic(dom[0])
    roofline = {"kernel": dom[0], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes": dom[2],
                "kernel_ms": dom[1], "per_visit_bytes": dom[3],
                "per_visit_GBs": dom[3] / (dom[1] * 1e-3) / 1e9 if dom[3] else None,
                # counted bandwidth: the profiled HBM bytes of one launch over the live kernel time
                "counted_GBs": traffic / (dom[1] * 1e-3) / 1e9 if traffic else None,
                "counted_frac": traffic / (dom[1] * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
                "traffic_over_algorithmic": traffic / dom[2] if traffic else None,
                "step_GBs": (BYTES_DILATE + BYTES_FILL) * mask.size / (ms_per_step * 1e-3) / 1e9,
                "kernel_source": kernel_sha(),
                "others": [{"kernel": c[0], "kernel_ms": c[1], "algorithmic_bytes": c[2],
                            "achieved": c[2] / (c[1] * 1e-3) / 1e9 if c[1] > 0 else None} for c in cand if c is not dom]}
    return {"ms_per_step": ms_per_step, "value": value, "kernels": kernels, "roofline": roofline,
            "outputs": outputs}


def next_ops(recon, torch, mask, steps, conn=8, h=20):
    """Reconstruction by erosion (marker I + h, capped: the dual of the headline
    marker), the h-dome and the regional maxima of the headline tile, each
    launched `steps` times back to back on fresh copies: throughput, kernel
    times, bit-exact parity of the last launch against the oracle, and the
    oracle's single-core time on the same tile."""
    import numpy as np
    dev = torch.device("cuda:0")
    up = np.minimum(mask.astype(np.int32) + h, 255).astype(np.uint8)
    d_mask = torch.from_numpy(mask).to(dev)
    ctx = recon.Recon(0, timing=1)
    stream = torch.cuda.current_stream()
    res = {"workload": "%dx%d nuclei-like tile, %d-conn, h %d; %d launches per op" % (
        mask.shape[0], mask.shape[1], conn, h, steps)}
    for op in ("erode", "hdome", "regional_max"):
        src = up if op == "erode" else mask
        bufs = [torch.from_numpy(src).to(dev) for _ in range(steps + 2)]
        torch.cuda.synchronize()

        def launch(b):
            if op == "erode":
                ctx.erode(b, d_mask, conn, stream)
            elif op == "hdome":
                ctx.hdome(b, h, conn, stream)
            else:
                ctx.regional_max(b, conn, stream)

        for b in bufs[:2]:
            launch(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in bufs[2:]:
            launch(b)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = [ctx.launch_times(back) for back in range(min(steps, 64))]
        st = ctx.last_stats()
        got = bufs[-1].cpu().numpy()
        call = {"erode": ("recon_erode", up, mask, conn), "hdome": ("hdome", mask, h, conn),
                "regional_max": ("regional_max", mask, conn)}[op]
        defer_check(("next_ops", op, "parity"), got, *call, rate_path=("next_ops", op, "oracle_single_core_Mpixel_s"),
                    px=mask.size)
        drain = sum(x["drain_ms"] for x in kt) / len(kt)
        visits = st["dense_visits"] + st["revisits"]
        res[op] = {"Mpixel_s": mask.size * steps / wall / 1e6, "ms_per_launch": wall * 1e3 / steps,
                   "revisit_drain_ms": drain, "launch_ms": sum(x["total_ms"] for x in kt) / len(kt),
                   "dense_visits": st["dense_visits"], "revisits": st["revisits"],
                   "revisit_drain_GBs": 3.0 * 32 * 256 * visits / (drain * 1e-3) / 1e9,
                   "oracle_single_core_Mpixel_s": None, "parity": None}
        log("%s: %.0f Mpixel/s (%.3f ms/launch)" % (op, res[op]["Mpixel_s"], res[op]["ms_per_launch"]))
        del bufs
    ctx.close()
    return res


def labelling(recon, torch, binary, steps, conn=8, lo=20, hi=1000):
    """Connected-component labelling (int32 labels) and the area filter of the
    headline tile's binary image (255 * (I > 120)), each launched `steps` times
    back to back: throughput, per-launch time from events on the launch stream,
    bit-exact parity of the last launch against the oracle, the oracle's
    single-core rate."""
    import numpy as np
    dev = torch.device("cuda:0")
    d_img = torch.from_numpy(binary).to(dev)
    planes = [torch.empty(binary.shape, dtype=torch.int32, device=dev) for _ in range(2)]
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    ctx = recon.Recon(0)
    stream = torch.cuda.current_stream()
    res = {"workload": "%dx%d binary nuclei tile (I > 120), %d-conn; area filter [%d, %d]; %d launches each" % (
        binary.shape[0], binary.shape[1], conn, lo, hi, steps)}
    for op in ("label", "area_threshold"):
        bufs = [d_img.clone() for _ in range(steps + 2)] if op == "area_threshold" else None

        def launch(s):
            if op == "label":
                ctx.label(d_img, planes[s % 2], conn, count, stream)
            else:
                ctx.area_threshold(bufs[s], lo, hi, conn, stream)

        for s in range(2):
            launch(s)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for s in range(steps):
            launch(2 + s)
            ev[s + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = [ev[s].elapsed_time(ev[s + 1]) for s in range(steps)]
        if op == "label":
            got = (planes[(2 + steps - 1) % 2].cpu().numpy(), int(count.item()))
            call = ("label", binary, conn)
        else:
            got = bufs[-1].cpu().numpy()
            call = ("area_threshold", binary, lo, hi, conn)
        defer_check(("labelling", op, "parity"), got, *call,
                    rate_path=("labelling", op, "oracle_single_core_Mpixel_s"), px=binary.size)
        # algorithmic bytes: read the image, write the int32 labels (5 B/px);
        # the area filter reads and writes the image (2 B/px)
        bpp = 5.0 if op == "label" else 2.0
        res[op] = {"Mpixel_s": binary.size * steps / wall / 1e6, "ms_per_launch": wall * 1e3 / steps,
                   "launch_ms_median": float(np.median(per)), "algorithmic_GBs": bpp * binary.size /
                   (float(np.median(per)) * 1e-3) / 1e9, "oracle_single_core_Mpixel_s": None, "parity": None}
        if op == "label":
            res[op]["components"] = int(count.item())
        log("%s: %.0f Mpixel/s (%.3f ms/launch)" % (op, res[op]["Mpixel_s"], res[op]["ms_per_launch"]))
        del bufs
    ctx.close()
    return res


def distance(recon, torch, binary, steps, conn=8):
    """Exact distance transform (int32 squared distances) and Pre-Watershed
    markers of the headline tile's binary image, each launched `steps` times
    back to back: throughput, per-launch time from events on the launch
    stream, bit-exact parity of the last launch against the oracle, the
    oracle's single-core rate."""
    import numpy as np
    dev = torch.device("cuda:0")
    d_img = torch.from_numpy(binary).to(dev)
    planes = [torch.empty(binary.shape, dtype=torch.int32, device=dev) for _ in range(2)]
    ctx = recon.Recon(0)
    stream = torch.cuda.current_stream()
    res = {"workload": "%dx%d binary nuclei tile (I > 120); markers %d-conn; %d launches each" % (
        binary.shape[0], binary.shape[1], conn, steps)}
    for op in ("distance", "pre_watershed"):
        bufs = [d_img.clone() for _ in range(steps + 2)] if op == "pre_watershed" else None

        def launch(s):
            if op == "distance":
                ctx.distance(d_img, planes[s % 2], stream)
            else:
                ctx.pre_watershed(bufs[s], conn, stream)

        for s in range(2):
            launch(s)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for s in range(steps):
            launch(2 + s)
            ev[s + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = [ev[s].elapsed_time(ev[s + 1]) for s in range(steps)]
        if op == "distance":
            defer_check(("distance", op, "parity"), planes[(2 + steps - 1) % 2].cpu().numpy(), "distance2", binary,
                        rate_path=("distance", op, "oracle_single_core_Mpixel_s"), px=binary.size)
        else:
            defer_check(("distance", op, "parity"), bufs[-1].cpu().numpy(), "pre_watershed", binary, conn,
                        rate_path=("distance", op, "oracle_single_core_Mpixel_s"), px=binary.size)
        # algorithmic bytes: read the image, write int32 distances (5 B/px);
        # the markers read and write the image (2 B/px)
        bpp = 5.0 if op == "distance" else 2.0
        res[op] = {"Mpixel_s": binary.size * steps / wall / 1e6, "ms_per_launch": wall * 1e3 / steps,
                   "launch_ms_median": float(np.median(per)),
                   "algorithmic_GBs": bpp * binary.size / (float(np.median(per)) * 1e-3) / 1e9,
                   "oracle_single_core_Mpixel_s": None, "parity": None}
        log("%s: %.0f Mpixel/s (%.3f ms/launch)" % (op, res[op]["Mpixel_s"], res[op]["ms_per_launch"]))
        del bufs
    ctx.close()
    return res


def batch_roofline(name, px, launch_ms):
    """Roofline of a batched launch: the method's bytes (3 B/px per reconstruction)
    over the launch, and the counted HBM bytes of its revisit kernel when the
    committed counter summary covers this section on the current kernels."""
    alg = BYTES_DILATE * px
    achieved = alg / (launch_ms * 1e-3) / 1e9
    traffic = committed_traffic("revisit_drain (%s)" % name)
    return {"bound": "hbm", "algorithmic_bytes": alg, "launch_ms": launch_ms, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_over_algorithmic": traffic / alg if traffic else None,
            "counted_GBs_over_launch": traffic / (launch_ms * 1e-3) / 1e9 if traffic else None}


def batched_vs_per_tile(recon, torch, ctx_cfg, n_tiles, size, workers, spiral_size, per_tile=True):
    """The 64-tile workload: one batched graph launch of all tiles against the
    same tiles as plain per-tile calls; also the 56 nuclei tiles alone and the 8
    spiral corridors alone as batched launches, so that the nuclei tiles'
    batched rate and the spirals' makespan are reported apart."""
    t0 = time.perf_counter()
    batch = make_batch(n_tiles, size, workers, spiral_size)
    log("batch: generated %d tiles in %.1f s" % (n_tiles, time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    masks = [torch.from_numpy(b[2]).to(dev) for b in batch]
    pristine = [torch.from_numpy(b[1]).to(dev) for b in batch]
    kinds = [b[0] for b in batch]
    px_of = lambda idx: sum(masks[i].numel() for i in idx)
    every = list(range(n_tiles))
    nuclei = [i for i in every if kinds[i] == "nuclei"]
    spirals = [i for i in every if kinds[i] == "spiral"]
    res = {"tiles": n_tiles, "tile": [size, size], "spirals": len(spirals),
           "spiral_tile": [spiral_size, spiral_size], "pixels": px_of(every)}
    # the autotuner's block rows, queue capacity and scan rounds for these tiles
    # (every tile has one size and 8-connectivity; knobs given on the command
    # line win), used by the batched launches and the per-tile calls alike
    from paper_1209_3332_amd import tune
    cache = tune.load_cache()
    knobs = tune.config_for(cache, size, size, 8)
    ctx_cfg = dict(ctx_cfg)
    for k in ("block_rows", "queue_capacity", "scan_rounds"):
        ctx_cfg.setdefault(k, knobs[k])
    res.update({"tuned": bool(cache), "block_rows": ctx_cfg["block_rows"],
                "queue_capacity": ctx_cfg["queue_capacity"], "scan_rounds": ctx_cfg["scan_rounds"]})
    with recon.Recon(0, **ctx_cfg) as ctx:
        stream = torch.cuda.current_stream()

        def batched(idx):
            # one graph replay over the tiles idx (the second of two runs is timed)
            for rep in range(2):
                work = {i: pristine[i].clone() for i in idx}
                torch.cuda.synchronize()
                t = time.perf_counter()
                ctx.batch([{"op": "dilate", "image": work[i], "mask": masks[i], "conn": 8} for i in idx], stream)
                st = ctx.last_stats()
                torch.cuda.synchronize()
                wall = time.perf_counter() - t
            return work, {"Mpixel_s": px_of(idx) / wall / 1e6, "ms": wall * 1e3, "launch_ms": st["total_ms"],
                          "revisits": st["revisits"], "component_tasks": st["component_tasks"]}

        work, res["batched"] = batched(every)
        res["roofline"] = batch_roofline("64-tile batch", px_of(every), res["batched"]["launch_ms"])
        # a spiral corridor's reconstruction is its mask; nuclei tiles go to the oracle leg
        res["spirals_equal_mask"] = all(torch.equal(work[i], masks[i]) for i in spirals)
        res["parity_checked_tiles"] = [nuclei[j] for j in sorted({0, len(nuclei) // 3, 2 * len(nuclei) // 3,
                                                                   len(nuclei) - 1})] if nuclei else []
        res["parity_ok"] = None
        for i in res["parity_checked_tiles"]:
            defer_check(("batched_vs_per_tile", "parity_ok"), work[i].cpu().numpy(), "recon_dilate", batch[i][1],
                        batch[i][2], 8)
        del work
        if nuclei and spirals:
            res["batched_nuclei_only"] = batched(nuclei)[1]
            w_s, res["batched_spirals_only"] = batched(spirals)
            res["batched_spirals_only"]["makespan_ms"] = res["batched_spirals_only"]["ms"]
            res["spirals_equal_mask"] = res["spirals_equal_mask"] and all(torch.equal(w_s[i], masks[i])
                                                                           for i in spirals)
            del w_s
        if not per_tile:
            return res
        # per-tile: the same tiles as plain calls, one after another
        work = [p.clone() for p in pristine]
        torch.cuda.synchronize()
        lat = []
        t = time.perf_counter()
        for w, m in zip(work, masks):
            ctx.dilate(w, m, 8, stream)
            lat.append(ctx.last_stats()["total_ms"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        nuc = [l for l, k in zip(lat, kinds) if k == "nuclei"]
        spi = [l for l, k in zip(lat, kinds) if k == "spiral"]
        res["per_tile"] = {"Mpixel_s": px_of(every) / wall / 1e6, "ms": wall * 1e3,
                           "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                                          "nuclei_p50": percentile(nuc, 50), "nuclei_p99": percentile(nuc, 99),
                                          "spiral_max": max(spi) if spi else None}}
        res["spirals_equal_mask"] = res["spirals_equal_mask"] and all(torch.equal(work[i], masks[i])
                                                                       for i in spirals)
        if nuc:
            res["per_tile"]["nuclei_Mpixel_s"] = px_of(nuclei) / (sum(nuc) * 1e-3) / 1e6
        res["batched_over_per_tile"] = res["batched"]["Mpixel_s"] / res["per_tile"]["Mpixel_s"]
    return res


def _gen_uneven(args):
    import synth
    i, h, w, hv, config = args
    mask = synth.scaled_config1_tile(h, w, synth.seed_for(config, i))
    return i, synth.hdome_marker(mask, hv), mask


def uneven_pool(n_tiles, config, workers):
    """Tiles of the uneven workload (sides from {512, ..., 4096}, conn 4 or 8, h in [10, 40])."""
    import multiprocessing as mp
    import synth
    shapes = synth.config4_shapes(n_tiles, synth.seed_for(config, 999_999))
    out = [None] * n_tiles
    with mp.get_context("fork").Pool(workers) as pool:
        for i, marker, mask in pool.imap_unordered(_gen_uneven, [(i, h, w, hv, config)
                                                                  for i, (h, w, _, hv) in enumerate(shapes)]):
            out[i] = (marker, mask, shapes[i][2])
    return out


def uneven_batched_vs_per_tile(recon, torch, n_tiles, workers, per_tile_legs=True):
    """The uneven batch as one autotuned graph launch vs as plain per-tile calls."""
    from paper_1209_3332_amd import tune
    t0 = time.perf_counter()
    tiles = uneven_pool(n_tiles, 4, workers)
    log("uneven batch: generated %d tiles in %.1f s" % (n_tiles, time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    masks = [torch.from_numpy(m).to(dev) for _, m, _ in tiles]
    pristine = [torch.from_numpy(j).to(dev) for j, _, _ in tiles]
    conns = [c for _, _, c in tiles]
    px = sum(m.numel() for m in masks)
    cache = tune.load_cache()
    bh, qcap, tuned = tune.tuned_batch(cache, [{"op": "dilate", "image": p, "mask": m, "conn": c}
                                              for p, m, c in zip(pristine, masks, conns)])
    res = {"tiles": n_tiles, "pixels": px, "tuned": bool(cache), "block_rows": bh, "queue_capacity": qcap}
    stream = torch.cuda.current_stream()
    with recon.Recon(0, block_rows=bh, queue_capacity=qcap, timing=1) as ctx:
        for rep in range(3):
            work = [p.clone() for p in pristine]
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.batch([dict(tk, image=w) for tk, w in zip(tuned, work)], stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
        st = ctx.last_stats()
        res["batched"] = {"Mpixel_s": px / wall / 1e6, "ms": wall * 1e3, "launch_ms": st["total_ms"],
                          "queue_overflows": st["queue_overflows"], "queue_spills": st["queue_spills"],
                          "revisits": st["revisits"], "reruns": st["reruns"], "dense_visits": st["dense_visits"]}
        res["roofline"] = batch_roofline("uneven batch", px, st["total_ms"])
        # parity on a stratified sample: two tiles of every size bucket and connectivity
        strata = {}
        for i, (j, m, c) in enumerate(tiles):
            strata.setdefault((tune.bucket_of(*m.shape), c), []).append(i)
        picks = sorted(i for idx in strata.values() for i in (idx[0], idx[-1]))
        res["parity_checked_tiles"] = sorted(set(picks))
        res["parity_strata"] = sorted("%s/conn%d" % k for k in strata)
        res["parity_ok"] = None
        for i in res["parity_checked_tiles"]:
            defer_check(("uneven_batched_vs_per_tile", "parity_ok"), work[i].cpu().numpy(), "recon_dilate",
                        tiles[i][0], tiles[i][1], conns[i])

    def per_tile(tuned_calls):
        """256 plain launches, one tile each: with the library defaults, or with
        each tile's own tuned knobs (a context per tuned block height, the
        tile's scan rounds and queue capacity as a one-task launch)."""
        ctxs = {}
        try:
            for rep in range(2):
                work = [p.clone() for p in pristine]
                torch.cuda.synchronize()
                t = time.perf_counter()
                for w, m, c, tk in zip(work, masks, conns, tuned):
                    if tuned_calls:
                        tb = tune.config_for(cache, *m.shape, c)["block_rows"]
                        if tb not in ctxs:
                            ctxs[tb] = recon.Recon(0, block_rows=tb, queue_capacity=qcap, timing=1)
                        ctxs[tb].batch([dict(tk, image=w)], stream)
                    else:
                        if None not in ctxs:
                            ctxs[None] = recon.Recon(0, timing=1)
                        ctxs[None].dilate(w, m, c, stream)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t
        finally:
            for cx in ctxs.values():
                cx.close()
        return {"Mpixel_s": px / wall / 1e6, "ms": wall * 1e3}

    if not per_tile_legs:
        return res
    res["per_tile"] = per_tile(False)
    res["per_tile_tuned"] = per_tile(True)
    res["batched_over_per_tile"] = res["batched"]["Mpixel_s"] / res["per_tile"]["Mpixel_s"]
    res["batched_over_per_tile_tuned"] = res["batched"]["Mpixel_s"] / res["per_tile_tuned"]["Mpixel_s"]
    return res


def serving(recon, torch, rates, seconds, pool_tiles, workers):
    """Poisson arrivals of uneven tiles (host-pinned pool) at each rate: upload,
    submit (retrying while admission is full), poll; latency = arrival to
    completion seen by poll, upload included.  Every 100th result is kept for
    the oracle leg."""
    import numpy as np
    pool = uneven_pool(pool_tiles, 5, workers)
    pinned = [(torch.from_numpy(j).pin_memory(), torch.from_numpy(m).pin_memory(), c) for j, m, c in pool]
    dev = torch.device("cuda:0")
    copy_stream = torch.cuda.Stream()
    rng = np.random.default_rng(5)
    out = []
    with recon.Recon(0) as ctx:
        for rate in rates:
            arrivals = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * seconds * 1.5) + 16))
            arrivals = arrivals[arrivals < seconds]
            picks = rng.integers(0, pool_tiles, size=len(arrivals))
            inflight, lat, sampled, again = [], [], [], 0
            px = 0
            t0 = time.perf_counter()
            k = 0

            def reap():
                still = []
                for tk, t_arr, buf, idx, n in inflight:
                    if ctx.poll(tk):
                        lat.append((time.perf_counter() - t0 - t_arr) * 1e3)
                        if n % 100 == 0:
                            sampled.append((buf[0].cpu().numpy(), idx))
                    else:
                        still.append((tk, t_arr, buf, idx, n))
                inflight[:] = still

            while k < len(arrivals) or inflight:
                now = time.perf_counter() - t0
                if k < len(arrivals) and now >= arrivals[k]:
                    j, m, c = pinned[picks[k]]
                    with torch.cuda.stream(copy_stream):
                        dj = j.to(dev, non_blocking=True)
                        dm = m.to(dev, non_blocking=True)
                    copy_stream.synchronize()
                    while True:
                        try:
                            tk = ctx.submit("dilate", dj, dm, c)
                            break
                        except recon.ReconAgain:
                            again += 1
                            reap()
                    inflight.append((tk, arrivals[k], (dj, dm), int(picks[k]), k))
                    px += dj.numel()
                    k += 1
                else:
                    reap()
            wall = time.perf_counter() - t0
            out.append({"rate_tiles_s": rate, "requests": len(arrivals), "tiles_s": len(arrivals) / wall,
                        "Mpixel_s": px / wall / 1e6, "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                        "admission_retries": again, "sampled": len(sampled), "checked": 0, "mismatches": 0})
            for got, idx in sampled:
                defer_check(("serving", len(out) - 1, "mismatches"), got, "recon_dilate", *pool[idx])
            log("serving at %d tiles/s: %.0f tiles/s done, p50 %.2f ms, p99 %.2f ms, %d results kept for the oracle" % (
                rate, out[-1]["tiles_s"], out[-1]["p50_ms"] or 0, out[-1]["p99_ms"] or 0, len(sampled)))
        ctx.serve_stop()
    return out


def _gen_pipe_tile(args):
    import synth
    i, size = args
    return i, synth.config2_tile(seed=synth.seed_for(6, i), size=size,
                                 n_gauss=round(3000 * size * size / 4096 ** 2))[1]


PIPE_IN = {"hdome": 1, "fill_holes": 1, "area_threshold": 1, "markers": 1, "label": 1}    # bytes/px read
PIPE_OUT = {"hdome": 1, "fill_holes": 1, "area_threshold": 1, "markers": 1, "label": 4}   # bytes/px written


def pipeline(recon, torch, n_tiles, size, window, cpu_workers, workers, windows=(), io_threads=2, h=20, conn=8,
             lo=20, hi=1000):
    """The co-scheduled tile pipeline (hdome -> fill-holes -> area filter ->
    {Pre-Watershed markers, labels}) on n_tiles nuclei-like tiles from host
    memory: the GPU alone, then the GPU beside cpu_workers CPU workers under
    FCFS and PATS, without and with data locality, and PATS with the CPU workers
    kept off the operations a core would take too long on, and the GPU manager
    keeping two instances enqueued at once and running up to 8 ready h-dome or
    fill-holes instances in one launch, alone and beside the CPU workers.
    Speedup estimates
    come from a calibration on one tile (each operation's CPU variant against
    its GPU variant, computation only); every run's outputs are compared byte
    for byte with the GPU-only run's, and two tiles with the oracle."""
    import multiprocessing as mp
    import numpy as np
    t0 = time.perf_counter()
    tiles = [None] * n_tiles
    with mp.get_context("fork").Pool(workers) as pool:
        for i, img in pool.imap_unordered(_gen_pipe_tile, [(i, size) for i in range(n_tiles)]):
            tiles[i] = img
    log("pipeline: generated %d tiles in %.1f s" % (n_tiles, time.perf_counter() - t0))
    ops = list(recon.PIPE_OPS)
    base = dict(conn=conn, h=h, area_min=lo, area_max=hi, io_threads=io_threads)
    # calibration: CPU variants on one tile, one core
    cpu_ms = {}
    x = tiles[0]
    cfg1 = recon.pipe_config(**base)
    for op in ops:
        src = x if op in ("hdome", "fill_holes", "area_threshold") else a_img
        t1 = time.perf_counter()
        y = recon.recon_pipeline_host_op(op, src, cfg1)
        cpu_ms[op] = (time.perf_counter() - t1) * 1e3
        if op in ("hdome", "fill_holes", "area_threshold"):
            x = y
        if op == "area_threshold":
            a_img = y
    res = {"tiles": n_tiles, "tile": [size, size], "pixels": n_tiles * size * size, "window": window,
           "cpu_workers": cpu_workers, "io_threads": io_threads, "gpus": 1, "conn": conn, "h": h, "area": [lo, hi]}
    # output buffers reused by every run (written once here, so that no run
    # pays the first touch of fresh host pages)
    bufs = recon.pipe_outputs(tiles)
    for o in bufs:
        for a in o.values():
            a.fill(0)

    def poison():
        # before each run: a first row no correct run leaves (objects and
        # markers are 0 / 255, labels >= 0), so a tile a run did not write shows
        for o in bufs:
            o["objects"][0, :] = 77
            o["markers"][0, :] = 77
            o["labels"][0, :] = -7
    with recon.Recon(0) as ctx:
        # GPU variants on the same tile (3 copies, the last two counted)
        _, st = recon.recon_pipeline_run(ctx.ctx, [tiles[0]], recon.pipe_config(cpu_workers=0, window=1, **base))
        _, st = recon.recon_pipeline_run(ctx.ctx, [tiles[0]] * 2, recon.pipe_config(cpu_workers=0, window=1,
                                                                                      **base))
        gpu_ms = {op: st["busy_gpu_ms"][k] / max(1, st["ops_gpu"][k]) for k, op in enumerate(ops)}
        gbs = (st["upload_bytes"] + st["download_bytes"]) / max(st["transfer_ms"], 1e-6) / 1e6
        speedup = {op: cpu_ms[op] / max(gpu_ms[op], 1e-6) for op in ops}
        xfer = {op: (PIPE_IN[op] + PIPE_OUT[op]) * size * size / (gbs * 1e6) for op in ops}   # ms at gbs GB/s
        impact = {op: xfer[op] / (xfer[op] + gpu_ms[op]) for op in ops}
        res["calibration"] = {"cpu_ms": cpu_ms, "gpu_ms": gpu_ms, "speedup": speedup,
                              "transfer_GBs": gbs, "transfer_impact": impact}
        log("pipeline calibration: speedups " + ", ".join("%s %.0f" % (o, speedup[o]) for o in ops))
        runs = [("gpu_only", dict(policy="pats", cpu_workers=0, data_locality=True)),
                ("gpu_only_prefetch", dict(policy="pats", cpu_workers=0, data_locality=True, prefetch=True)),
                ("fcfs", dict(policy="fcfs", cpu_workers=cpu_workers, data_locality=False)),
                ("fcfs_dl", dict(policy="fcfs", cpu_workers=cpu_workers, data_locality=True)),
                ("pats", dict(policy="pats", cpu_workers=cpu_workers, data_locality=False)),
                ("pats_dl", dict(policy="pats", cpu_workers=cpu_workers, data_locality=True)),
                ("pats_dl_cutoff", None),
                ("pats_dl_guard", dict(policy="pats", cpu_workers=cpu_workers, data_locality=True, cpu_guard=True)),
                ("pats_dl_guard_prefetch", dict(policy="pats", cpu_workers=cpu_workers, data_locality=True,
                                                cpu_guard=True, prefetch=True)),
                # the GPU manager keeping two instances enqueued (the next one is
                # chosen and enqueued while the previous one runs)
                ("gpu_only_prefetch_inflight2", dict(policy="pats", cpu_workers=0, data_locality=True,
                                                     prefetch=True, gpu_inflight=2)),
                ("pats_dl_guard_prefetch_inflight2", dict(policy="pats", cpu_workers=cpu_workers,
                                                          data_locality=True, cpu_guard=True, prefetch=True,
                                                          gpu_inflight=2)),
                # and running up to 8 ready h-dome or fill-holes instances in one launch
                ("gpu_only_prefetch_inflight2_batch8", dict(policy="pats", cpu_workers=0, data_locality=True,
                                                            prefetch=True, gpu_inflight=2, gpu_batch=8)),
                ("pats_dl_guard_prefetch_inflight2_batch8", dict(policy="pats", cpu_workers=cpu_workers,
                                                                 data_locality=True, cpu_guard=True,
                                                                 prefetch=True, gpu_inflight=2, gpu_batch=8)),
                # the GPU alone needs no CPU workers: their cores copy tiles in and out instead
                ("gpu_only_prefetch_inflight2_batch8_io8", dict(policy="pats", cpu_workers=0, data_locality=True,
                                                                prefetch=True, gpu_inflight=2, gpu_batch=8,
                                                                io_threads=2 * io_threads))]
        ref = None
        res["runs"] = {}
        for name, kw in runs:
            if kw is None:
                # CPU workers may take only the operations whose CPU time is at
                # most a quarter of the GPU-only makespan of this batch
                m = res["runs"]["gpu_only"]["makespan_ms"]
                ok_ops = [o for o in ops if cpu_ms[o] <= m / 4]
                limit = max((speedup[o] for o in ok_ops), default=0.5 * min(speedup.values()))
                kw = dict(policy="pats", cpu_workers=cpu_workers, data_locality=True, cpu_max_speedup=limit)
                res["cutoff"] = {"cpu_max_speedup": limit, "cpu_ops": ok_ops}
            cfg = recon.pipe_config(window=window, speedup=speedup, transfer_impact=impact, gpu_ms=gpu_ms,
                                    **dict(base, **kw))
            poison()
            outs, st = recon.recon_pipeline_run(ctx.ctx, tiles, cfg, outputs=bufs)
            r = {"makespan_ms": st["makespan_ms"], "tiles_s": n_tiles / (st["makespan_ms"] * 1e-3),
                 "Mpixel_s": res["pixels"] / (st["makespan_ms"] * 1e-3) / 1e6,
                 "ops_cpu": dict(zip(ops, st["ops_cpu"])), "ops_gpu": dict(zip(ops, st["ops_gpu"])),
                 "uploads": st["uploads"], "downloads": st["downloads"],
                 "transfer_GB": (st["upload_bytes"] + st["download_bytes"]) / 1e9,
                 "transfer_ms": st["transfer_ms"], "io_ms": st["io_ms"], "policy": kw["policy"],
                 "data_locality": kw["data_locality"], "prefetch": bool(kw.get("prefetch")),
                 "gpu_inflight": max(1, kw.get("gpu_inflight", 1)), "gpu_batch": max(1, kw.get("gpu_batch", 1)),
                 "io_threads": kw.get("io_threads", io_threads)}
            if ref is None:
                ref = [{k: (v.copy() if hasattr(v, "copy") else v) for k, v in o.items()} for o in outs]
                for i in (0, n_tiles - 1):
                    defer_check(("pipeline", "parity_tiles_%d" % i), ref[i], "pipeline_chain", tiles[i], h, conn,
                                lo, hi)
                    res["parity_tiles_%d" % i] = None
            else:
                r["same_as_gpu_only"] = all(
                    np.array_equal(o[k], q[k]) for o, q in zip(outs, ref) for k in ("objects", "markers", "labels")
                ) and all(o["count"] == q["count"] for o, q in zip(outs, ref))
            res["runs"][name] = r
            log("pipeline %s: %.1f ms (%.1f tiles/s), CPU ops %s" % (
                name, r["makespan_ms"], r["tiles_s"], sum(st["ops_cpu"])))
            del outs
        # the window sweep (Table 2's experiment): FCFS and PATS with data locality
        res["window_sweep"] = {}
        for w in windows:
            for pol in ("fcfs", "pats"):
                cfg = recon.pipe_config(policy=pol, cpu_workers=cpu_workers, window=w, data_locality=True,
                                        speedup=speedup, transfer_impact=impact, **base)
                poison()
                outs, st = recon.recon_pipeline_run(ctx.ctx, tiles, cfg, outputs=bufs)
                same = all(np.array_equal(o[k], q[k]) for o, q in zip(outs, ref)
                           for k in ("objects", "markers", "labels"))
                res["window_sweep"]["%s_dl/w%d" % (pol, w)] = {
                    "makespan_ms": st["makespan_ms"], "cpu_ops": sum(st["ops_cpu"]), "same_as_gpu_only": same}
                log("pipeline %s_dl window %d: %.1f ms" % (pol, w, st["makespan_ms"]))
                del outs
        # against the better of the two GPU-only runs with one instance at a time
        g = min(res["runs"]["gpu_only"]["makespan_ms"], res["runs"]["gpu_only_prefetch"]["makespan_ms"])
        res["speedup_over_gpu_only"] = {k: g / v["makespan_ms"] for k, v in res["runs"].items()}
        res["pats_over_fcfs"] = res["runs"]["fcfs"]["makespan_ms"] / res["runs"]["pats"]["makespan_ms"]
        res["pats_dl_over_fcfs_dl"] = res["runs"]["fcfs_dl"]["makespan_ms"] / res["runs"]["pats_dl"]["makespan_ms"]
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--batch-tiles", type=int, default=64, help="0 skips the batched-vs-per-tile comparison")
    ap.add_argument("--spiral-size", type=int, default=4096, help="side of the spiral-corridor tiles of the batch")
    ap.add_argument("--uneven-tiles", type=int, default=256, help="0 skips the uneven autotuned batch")
    ap.add_argument("--serve-rates", default="50,100,200,500,1000,2000",
                    help="Poisson arrival rates (tiles/s) of the serving run; empty skips it")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="seconds of arrivals per rate")
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--next-ops-steps", type=int, default=10,
                    help="launches per op of erosion / h-dome / regional maxima on the tile (0 skips)")
    ap.add_argument("--label-steps", type=int, default=10,
                    help="launches of labelling and of the area filter on the binary tile (0 skips)")
    ap.add_argument("--distance-steps", type=int, default=10,
                    help="launches of the distance transform and of the Pre-Watershed markers (0 skips)")
    ap.add_argument("--step-mode", choices=("batched", "plain"), default="batched",
                    help="headline step: both operations in one batched launch, or two plain calls")
    ap.add_argument("--plain-steps", type=int, default=20,
                    help="with --step-mode batched: also time the step as plain calls (0 skips)")
    ap.add_argument("--block-rows", type=int, default=0)
    ap.add_argument("--scan-rounds", type=int, default=0)
    ap.add_argument("--queue", type=int, default=0)
    ap.add_argument("--drain-budget", type=int, default=0, help="context knob (0 = library default)")
    ap.add_argument("--binary-drain-budget", type=int, default=0, help="context knob (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-tile", action="store_true",
                    help="batch sections time the batched launches only (for counter runs)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device 5 times (counter calibration) and exit")
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    ap.add_argument("--pipeline-tiles", type=int, default=64,
                    help="tiles of the co-scheduled pipeline section (0 skips it)")
    ap.add_argument("--pipeline-window", type=int, default=16)
    # one core for the GPU manager thread and four for the I/O threads, the rest run CPU variants
    ap.add_argument("--pipeline-cpu-workers", type=int, default=max(1, min(16, len(os.sched_getaffinity(0))) - 5))
    ap.add_argument("--pipeline-io-threads", type=int, default=4)
    ap.add_argument("--pipeline-windows", default="8,32",
                    help="extra window sizes for the FCFS / PATS (with DL) sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the reconstruction shards by tile with no communication, "
              "and this build measures the single-GPU path only (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        a = torch.empty(args.copy_probe, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 5}))
        return

    import paper_1209_3332_amd as recon
    import synth

    marker, mask, binary = synth.config2_tile(size=args.size, n_gauss=round(3000 * args.size ** 2 / 4096 ** 2))
    cfg = dict(timing=1)
    if args.block_rows:
        cfg["block_rows"] = args.block_rows
    if args.scan_rounds:
        cfg["scan_rounds"] = args.scan_rounds
    if args.queue:
        cfg["queue_capacity"] = args.queue
    if args.drain_budget:
        cfg["drain_budget"] = args.drain_budget
    if args.binary_drain_budget:
        cfg["binary_drain_budget"] = args.binary_drain_budget
    main = headline(recon, torch, cfg, marker, mask, binary, args.steps, args.warmup, args.step_mode)
    ms_per_step, value, kernels, roofline = (main[k] for k in ("ms_per_step", "value", "kernels", "roofline"))
    parity = {"dilate": None, "fill_holes": None}   # filled by the oracle leg
    how = ("both in one batched launch per tile" if args.step_mode == "batched"
           else "as two plain per-tile launches")
    out = {"metric": METRIC, "value": value, "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "one uint8 %dx%d nuclei-like tile: 8-conn reconstruction (marker I-20) + "
                                  "8-conn fill-holes of I>120, %s" % (args.size, args.size, how),
                      "pixels_per_step": 2 * mask.size, "block_rows": cfg.get("block_rows", 32)},
           "kernels": kernels, "roofline": roofline, "parity": parity}
    defer_check(("parity", "dilate"), main["outputs"]["dilate"], "recon_dilate", marker, mask, 8)
    defer_check(("parity", "fill_holes"), main["outputs"]["fill_holes"], "fill_holes", binary, 8)
    if args.step_mode == "batched" and args.plain_steps:
        # the same step as two plain per-tile calls, with each operation's kernels
        plain = headline(recon, torch, cfg, marker, mask, binary, args.plain_steps, args.warmup, "plain")
        out["plain_per_op"] = {k: plain[k] for k in ("ms_per_step", "value", "kernels")}
        out["plain_per_op"]["parity"] = {"dilate": None, "fill_holes": None}
        defer_check(("plain_per_op", "parity", "dilate"), plain["outputs"]["dilate"], "recon_dilate", marker, mask, 8)
        defer_check(("plain_per_op", "parity", "fill_holes"), plain["outputs"]["fill_holes"], "fill_holes", binary, 8)
        out["plain_per_op"]["roofline_dominant"] = {k: plain["roofline"][k] for k in
                                                    ("kernel", "achieved", "frac", "traffic", "kernel_ms")}
    if args.next_ops_steps:
        out["next_ops"] = next_ops(recon, torch, mask, args.next_ops_steps)
    if args.label_steps:
        out["labelling"] = labelling(recon, torch, binary, args.label_steps)
    if args.distance_steps:
        out["distance"] = distance(recon, torch, binary, args.distance_steps)
    if args.batch_tiles:
        out["batched_vs_per_tile"] = batched_vs_per_tile(recon, torch, {k: v for k, v in cfg.items()},
                                                         args.batch_tiles, args.size, args.workers,
                                                         args.spiral_size, per_tile=not args.no_per_tile)
        b = out["batched_vs_per_tile"]
        log("batch of %d: batched %.0f Mpixel/s vs per-tile %s Mpixel/s" % (
            args.batch_tiles, b["batched"]["Mpixel_s"], "%.0f" % b["per_tile"]["Mpixel_s"] if "per_tile" in b else "-"))
    if args.uneven_tiles:
        out["uneven_batched_vs_per_tile"] = uneven_batched_vs_per_tile(recon, torch, args.uneven_tiles, args.workers,
                                                                       per_tile_legs=not args.no_per_tile)
        u = out["uneven_batched_vs_per_tile"]
        log("uneven batch of %d: batched %.0f Mpixel/s vs per-tile %s Mpixel/s" % (
            args.uneven_tiles, u["batched"]["Mpixel_s"], "%.0f" % u["per_tile"]["Mpixel_s"] if "per_tile" in u else "-"))
    if args.serve_rates:
        rates = [int(r) for r in args.serve_rates.split(",") if r]
        out["serving"] = serving(recon, torch, rates, args.serve_seconds, args.serve_pool, args.workers)
    if args.pipeline_tiles:
        out["pipeline"] = pipeline(recon, torch, args.pipeline_tiles, args.size, args.pipeline_window,
                                   args.pipeline_cpu_workers, args.workers,
                                   windows=[int(w) for w in args.pipeline_windows.split(",") if w],
                                   io_threads=args.pipeline_io_threads)
    ok = True
    if not args.no_cpu_baseline:
        # the oracle leg: its rate on the host cores, then every deferred comparison
        out["cpu_baseline"] = cpu_baseline(marker, mask, binary)
        log("cpu baseline: %.1f Mpixel/s on %d cores" % (out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"]))
        ok = run_checks(out, args.workers)
        log("oracle checks: %d compared, %s" % (len(CHECKS), "all equal" if ok else "MISMATCH"))
    print(json.dumps(out), flush=True)
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
