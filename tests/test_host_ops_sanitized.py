"""The CPU variants of the tile pipeline (paper_1209_3332_amd/csrc/host_ops.cpp)
built with AddressSanitizer and UBSan (g++, host code only) and run on exact-size
allocations with padded pitches, on random images of many shapes (degenerate
ones included), for every operation; results against the oracle."""
import os
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("hostops") / "driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, os.path.join(HERE, "host_ops_san", "driver.cpp"),
                    os.path.join(ROOT, "paper_1209_3332_amd", "csrc", "host_ops.cpp")], check=True)
    return exe


def run(driver, tmp_path, op, img, conn=8, h=20, lo=20, hi=1000, planes=None):
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    data = np.concatenate([p.ravel() for p in planes]) if planes else img.ravel()
    src.write_bytes(np.ascontiguousarray(data, dtype=np.uint8).tobytes())
    r = subprocess.run([driver, str(op), str(conn), str(h), str(lo), str(hi), str(img.shape[0]), str(img.shape[1]),
                        str(src), str(dst)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    raw = dst.read_bytes()
    dt = np.int32 if op in (4, 6) else np.uint8
    return np.frombuffer(raw, dtype=dt).reshape(img.shape)


def images():
    rng = np.random.default_rng(4242)
    out = []
    for h, w in ((1, 1), (1, 9), (9, 1), (2, 3), (17, 33), (64, 5), (40, 257)):
        out.append(rng.integers(0, 256, size=(h, w), dtype=np.uint8))
        out.append(np.where(rng.random((h, w)) < 0.6, 255, 0).astype(np.uint8))
    out.append(synth.scaled_config1_tile(120, 170, synth.seed_for(9, 60)))
    out.append(np.zeros((5, 6), np.uint8))
    out.append(np.full((5, 6), 255, np.uint8))
    return out


@pytest.mark.parametrize("conn", [4, 8])
def test_host_ops_under_sanitizers(driver, tmp_path, oracle_mod, conn):
    rng = np.random.default_rng(conn)
    for img in images():
        assert np.array_equal(run(driver, tmp_path, 0, img, conn, h=25), oracle_mod.hdome(img, 25, conn))
        assert np.array_equal(run(driver, tmp_path, 1, img, conn), oracle_mod.fill_holes(img, conn))
        assert np.array_equal(run(driver, tmp_path, 2, img, conn, lo=2, hi=60),
                              oracle_mod.area_threshold(img, 2, 60, conn))
        assert np.array_equal(run(driver, tmp_path, 3, img, conn), oracle_mod.pre_watershed(img, conn))
        assert np.array_equal(run(driver, tmp_path, 4, img, conn), oracle_mod.label(img, conn)[0])
        assert np.array_equal(run(driver, tmp_path, 6, img, conn), oracle_mod.distance2(img))
        marker = np.minimum(img, rng.integers(0, 256, size=img.shape, dtype=np.uint8))
        assert np.array_equal(run(driver, tmp_path, 5, img, conn, planes=[marker, img]),
                              oracle_mod.recon_dilate(marker, img, conn))


def test_scheduler_under_thread_sanitizer(tmp_path):
    """The co-scheduling runtime with four CPU workers and three I/O threads,
    both policies, windows 1, 3 and 7, built with ThreadSanitizer (host code
    only; the GPU entry points are link stubs a CPU-only run never calls): no
    race report, and every tile equal to the CPU variants run in order."""
    exe = str(tmp_path / "pipeline_tsan")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-o", exe, os.path.join(HERE, "host_ops_san", "pipeline_tsan.cpp"),
                    os.path.join(ROOT, "paper_1209_3332_amd", "csrc", "pipeline.cpp"),
                    os.path.join(ROOT, "paper_1209_3332_amd", "csrc", "host_ops.cpp"),
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout, r.stderr[-2000:])
