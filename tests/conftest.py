import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU checks")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    """Key / value lines of a fixture under tests/golden ('#' comments);
    keys may repeat (a list of value strings per key, in file order)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            out.setdefault(key, []).append(rest)
    return out


def golden_small_fields():
    """(name, model, H, W, nbins, seed, width, p_min, p_max) of
    oracle_small_fields.txt (values as float arrays)."""
    import numpy as np
    g = read_golden("oracle_small_fields.txt")
    rows = []
    for case, pmin, pmax in zip(g["case"], g["p_min"], g["p_max"]):
        name, model, H, W, nb, seed, width = case.split()
        H, W = int(H), int(W)
        rows.append((name, int(model), H, W, int(nb), int(seed), float(width),
                     np.array([float.fromhex(v) for v in pmin.split()]).reshape(H, W),
                     np.array([float.fromhex(v) for v in pmax.split()]).reshape(H, W)))
    return rows
