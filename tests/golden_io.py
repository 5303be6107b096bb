"""Loading of the hand-derived fixtures under tests/golden/."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def num(v):
    """Fixture numbers are JSON numbers or short expressions like '1+1e-15'."""
    if isinstance(v, str):
        if "+" in v[1:]:
            a, b = v.split("+", 1)
            return float(a) + float(b)
        if "-" in v[1:]:
            i = v.index("-", 1)
            return float(v[:i]) - float(v[i + 1:])
        return float(v)
    return float(v)


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def graph_arrays(g):
    """(n, m, d, col_idx int32[n*d]) from a fixture's graph block."""
    n, m, d = g["n"], g["m"], g["d"]
    col = np.array(g["N"], dtype=np.int32).reshape(n * d)
    return n, m, d, col


def decode_cases():
    """(fixture name, graph, y, x, case) for every decode case in W*.json."""
    out = []
    for fn in sorted(os.listdir(GOLDEN)):
        if not fn.startswith("W"):
            continue
        fx = load(fn)
        for c in fx["cases"]:
            out.append((fx["name"], fx["graph"], np.array(fx["y"], float), np.array(fx["x"], float), c))
    return out
