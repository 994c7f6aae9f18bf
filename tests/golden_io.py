"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fig1_database():
    """Returns (D [n][m] uint8 with 0-based states, arity uint8[n])."""
    rows, arity = [], None
    with open(os.path.join(GOLDEN, "fig1_reconstructed.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("arity"):
                arity = np.array([int(x) for x in line.split()[1:]], dtype=np.uint8)
            else:
                rows.append([int(x) for x in line.split()])
    D = (np.array(rows, dtype=np.int64).T - 1).astype(np.uint8)   # 1-based -> 0-based
    return np.ascontiguousarray(D), arity


def fig1_expected():
    out = {}
    with open(os.path.join(GOLDEN, "fig1_expected.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key == "table":
                out[key] = np.array([int(v) for v in vals], dtype=np.int64)
            else:
                out[key] = float(vals[0])
    return out
