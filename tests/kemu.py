"""Driver for the host emulation of the HIP kernels (tests/kernel_emu).

The kernels' device code is compiled for the CPU against a stand-in HIP
header and run on emulated 64-lane waves, so that the scheduler and the pixel
logic can be checked against the oracle, and bounds-checked under
AddressSanitizer, without a GPU.
"""
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC_DIR = os.path.join(HERE, "kernel_emu")
CLANG = "/opt/rocm/llvm/bin/clang++"


def build(out_dir, sanitize=True):
    exe = os.path.join(out_dir, "kemu%s" % ("_asan" if sanitize else ""))
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-DKEMU_MAIN", "-I", SRC_DIR, "-o", exe,
           os.path.join(SRC_DIR, "emu.cpp"), "-lpthread"]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=undefined"]
    subprocess.run(cmd, check=True)
    return exe


OPS = {"dilate": 0, "fill_holes": 1, "erode": 2, "hdome": 3, "regional_max": 4}
TWO_PLANE = ("dilate", "erode")


def run(exe, tasks, bh=32, qcap=2048, scan_rounds=2, n_waves=4, watchdog_s=20.0, timeout=600, stop_after=0,
        test_fault=0, component=0, spill=0):
    """tasks: list of dicts {op, marker+mask (dilate, erode) or img (fill_holes,
    hdome, regional_max), conn, h (hdome)}.
    Returns (returncode, outputs, stdout+stderr)."""
    with tempfile.TemporaryDirectory() as d:
        lines = []
        for k, t in enumerate(tasks):
            two = t["op"] in TWO_PLANE
            img = np.ascontiguousarray(t["marker"] if two else t["img"], dtype=np.uint8)
            ip, mp, op = (os.path.join(d, "%d_%s.bin" % (k, s)) for s in ("img", "mask", "out"))
            img.tofile(ip)
            if two:
                np.ascontiguousarray(t["mask"], dtype=np.uint8).tofile(mp)
            else:
                mp = "-"
            lines.append("%d %d %d %d %d %s %s %s" % (OPS[t["op"]], t["conn"], t.get("h", 0),
                                                      img.shape[0], img.shape[1], ip, mp, op))
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1", KEMU_TEST_FAULT=str(int(test_fault)),
                   KEMU_COMPONENT=str(int(component)), KEMU_SPILL=str(int(spill)))
        p = subprocess.run([exe, str(bh), str(qcap), str(scan_rounds), str(n_waves), str(watchdog_s),
                            str(len(tasks)), str(stop_after)], input="\n".join(lines) + "\n", capture_output=True,
                           text=True, timeout=timeout, env=env)
        outs = []
        for k, t in enumerate(tasks):
            shape = (t["marker"] if t["op"] in TWO_PLANE else t["img"]).shape
            op = os.path.join(d, "%d_out.bin" % k)
            outs.append(np.fromfile(op, dtype=np.uint8).reshape(shape) if os.path.exists(op) else None)
        return p.returncode, outs, p.stdout + p.stderr


def run_label(exe, img, conn, min_area=0, max_area=1 << 40, n_waves=4, timeout=600):
    """Labelling and area filter of one image on the emulated kernels.
    Returns (returncode, labels int32, count, area-filtered uint8, log)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    h, w = img.shape
    with tempfile.TemporaryDirectory() as d:
        ip, lp, ap = (os.path.join(d, s) for s in ("img.bin", "lab.bin", "area.bin"))
        img.tofile(ip)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
        p = subprocess.run([exe, "label", str(conn), str(h), str(w), str(n_waves), str(min_area), str(max_area),
                            ip, lp, ap], capture_output=True, text=True, timeout=timeout, env=env)
        log = p.stdout + p.stderr
        if p.returncode != 0 or not os.path.exists(lp):
            return p.returncode, None, None, None, log
        count = int(log.split("count")[1].split()[0])
        return (p.returncode, np.fromfile(lp, np.int32).reshape(h, w), count,
                np.fromfile(ap, np.uint8).reshape(h, w), log)


def run_edt(exe, img, n_waves=3, timeout=600):
    """Distance transform of one image on the emulated kernels: (rc, dist2 int32, D8 uint8, log)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    h, w = img.shape
    with tempfile.TemporaryDirectory() as d:
        ip, dp, ep = (os.path.join(d, s) for s in ("img.bin", "d2.bin", "d8.bin"))
        img.tofile(ip)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
        p = subprocess.run([exe, "edt", str(h), str(w), str(n_waves), ip, dp, ep], capture_output=True, text=True,
                           timeout=timeout, env=env)
        log = p.stdout + p.stderr
        if p.returncode != 0 or not os.path.exists(dp):
            return p.returncode, None, None, log
        return p.returncode, np.fromfile(dp, np.int32).reshape(h, w), np.fromfile(ep, np.uint8).reshape(h, w), log
