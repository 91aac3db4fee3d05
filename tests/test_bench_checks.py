"""The benchmark's oracle leg (CPU only): deferred comparisons land in the
output line, a planted difference is reported, labelling compares labels and
count, and sampled serving results are counted."""
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_deferred_checks(oracle_mod):
    b = _bench()
    rng = np.random.default_rng(3)
    mask = rng.integers(0, 256, (40, 70)).astype(np.uint8)
    marker = np.maximum(mask.astype(np.int32) - 20, 0).astype(np.uint8)
    binary = np.where(mask > 120, 255, 0).astype(np.uint8)
    good = oracle_mod.recon_dilate(marker, mask, 8)
    bad = good.copy()
    bad[5, 7] ^= 1
    lab, n = oracle_mod.label(binary, 8)
    out = {"parity": {"dilate": None, "fill_holes": None}, "labelling": {"label": {"parity": None, "rate": None}},
           "serving": [{"checked": 0, "mismatches": 0}]}
    b.CHECKS.clear()
    b.defer_check(("parity", "dilate"), good, "recon_dilate", marker, mask, 8)
    b.defer_check(("parity", "fill_holes"), oracle_mod.fill_holes(binary, 8), "fill_holes", binary, 8)
    b.defer_check(("labelling", "label", "parity"), (lab, n), "label", binary, 8,
                  rate_path=("labelling", "label", "rate"), px=binary.size)
    b.defer_check(("serving", 0, "mismatches"), good, "recon_dilate", marker, mask, 8)
    b.defer_check(("serving", 0, "mismatches"), bad, "recon_dilate", marker, mask, 8)
    assert not b.run_checks(out)                    # the planted difference is seen
    assert out["parity"] == {"dilate": True, "fill_holes": True}
    assert out["labelling"]["label"]["parity"] is True and out["labelling"]["label"]["rate"] > 0
    assert out["serving"][0] == {"checked": 2, "mismatches": 1}
    b.CHECKS.clear()
    b.defer_check(("labelling", "label", "parity"), (lab, n + 1), "label", binary, 8)
    assert not b.run_checks(out) and out["labelling"]["label"]["parity"] is False   # a wrong count fails


def test_repeated_path_is_the_conjunction(oracle_mod):
    """Several sampled tiles report into one parity field: one bad tile makes it False."""
    b = _bench()
    rng = np.random.default_rng(4)
    mask = rng.integers(0, 256, (30, 50)).astype(np.uint8)
    marker = np.maximum(mask.astype(np.int32) - 20, 0).astype(np.uint8)
    good = oracle_mod.recon_dilate(marker, mask, 8)
    bad = good.copy()
    bad[3, 3] ^= 4
    out = {"batch": {"parity_ok": None}}
    b.CHECKS.clear()
    for got in (good, bad, good):
        b.defer_check(("batch", "parity_ok"), got, "recon_dilate", marker, mask, 8)
    assert not b.run_checks(out, workers=3)
    assert out["batch"]["parity_ok"] is False
    b.CHECKS.clear()
    out = {"batch": {"parity_ok": None}}
    for got in (good, good):
        b.defer_check(("batch", "parity_ok"), got, "recon_dilate", marker, mask, 8)
    assert b.run_checks(out) and out["batch"]["parity_ok"] is True


def test_pipeline_chain_check(oracle_mod):
    """The tile pipeline's outputs are checked against the oracle's chain of the
    same operations; a wrong marker pixel or count is reported."""
    b = _bench()
    import synth
    img = synth.scaled_config1_tile(96, 130, synth.seed_for(9, 40))
    a = oracle_mod.area_threshold(oracle_mod.fill_holes(oracle_mod.hdome(img, 20, 8), 8), 20, 1000, 8)
    lab, n = oracle_mod.label(a, 8)
    good = {"objects": a, "markers": oracle_mod.pre_watershed(a, 8), "labels": lab, "count": n}
    bad = dict(good, markers=good["markers"].copy())
    bad["markers"][3, 4] ^= 255
    out = {"pipeline": {"parity_tiles_0": None, "parity_tiles_1": None, "parity_tiles_2": None}}
    b.CHECKS.clear()
    b.defer_check(("pipeline", "parity_tiles_0"), good, "pipeline_chain", img, 20, 8, 20, 1000)
    b.defer_check(("pipeline", "parity_tiles_1"), bad, "pipeline_chain", img, 20, 8, 20, 1000)
    b.defer_check(("pipeline", "parity_tiles_2"), dict(good, count=n + 1), "pipeline_chain", img, 20, 8, 20, 1000)
    assert not b.run_checks(out)
    assert out["pipeline"] == {"parity_tiles_0": True, "parity_tiles_1": False, "parity_tiles_2": False}
