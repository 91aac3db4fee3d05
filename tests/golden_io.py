"""Reader for the hand-worked fixtures in tests/golden/*.txt.

Each file holds comment lines (``#``, the derivation and its citation),
``op:`` (dilate | fill_holes), ``conn:`` (one or more of 4 8) and matrices
introduced by ``mask:``, ``marker:``, ``img:`` and ``expect:``.
"""
import glob
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(path):
    case = {"name": os.path.splitext(os.path.basename(path))[0]}
    key = None
    rows = []

    def flush():
        if key is not None and rows:
            case[key] = np.array(rows, dtype=np.uint8)

    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("op:"):
                case["op"] = line.split(":", 1)[1].strip()
            elif line.startswith("conn:"):
                case["conns"] = [int(c) for c in line.split(":", 1)[1].split()]
            elif line.endswith(":"):
                flush()
                key, rows = line[:-1], []
            else:
                rows.append([int(v) for v in line.split()])
    flush()
    return case


def all_cases():
    return [load(p) for p in sorted(glob.glob(os.path.join(GOLDEN_DIR, "*.txt")))]
