"""Seeded synthetic instances for expander l0-decoding (inputs only).

The draws are done by ``l0gen.c`` (counter-based SplitMix64, so results do
not depend on thread count); this module compiles it on demand, wraps it with
ctypes and assembles :class:`Instance` objects.  Nothing here scores, selects
or updates anything: it serves the oracle and the GPU decoder alike as a
source of inputs.

Workload shapes follow the paper's synthetic experiments (Section 5): A with
d ones per column at rows drawn uniformly without replacement (footnote in
Section 1.1), x k-sparse with a uniform support and N(0,1) nonzeros (Section 5
preamble), or uniform +-1 nonzeros for the non-dissociated check.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "l0gen.c")
_LIB = os.path.join(_HERE, "libl0gen.so")

#: Base seed of every synthetic workload; instance i of workload c uses
#: ``SEED + 1000 * c + i``.
SEED = 150801256

VALUES_NORMAL = 0
VALUES_PM1 = 1


def build(force: bool = True) -> str:
    """Compile ``libl0gen.so`` next to its source with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-std=c11", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.l0gen_columns.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P]
        lib.l0gen_support.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, P]
        lib.l0gen_values.argtypes = [ctypes.c_uint64, ctypes.c_int64, P, ctypes.c_int32, P]
        lib.l0gen_measure.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                                      ctypes.c_int64, P, P, P, P]
        lib.l0gen_weights.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_double, P]
        for f in (lib.l0gen_columns, lib.l0gen_support, lib.l0gen_values, lib.l0gen_measure,
                  lib.l0gen_weights):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else None


def columns(seed: int, n: int, m: int, d: int) -> np.ndarray:
    """int32[n*d]: column j's d distinct rows at [j*d, j*d+d), ascending."""
    out = np.empty(n * d, dtype=np.int32)
    if _load().l0gen_columns(seed, n, m, d, _ptr(out)) != 0:
        raise ValueError(f"bad column arguments n={n} m={m} d={d}")
    return out


def permute_rows(col_idx: np.ndarray, d: int, seed: int) -> np.ndarray:
    """A copy of col_idx with each column's d rows in a seeded random order
    (the same graph A; only the order in which a column lists its rows
    changes)."""
    col = np.ascontiguousarray(col_idx, dtype=np.int32).reshape(-1, d)
    rng = np.random.Generator(np.random.PCG64(seed))
    order = np.argsort(rng.random(col.shape), axis=1, kind="stable")
    return np.take_along_axis(col, order, axis=1).reshape(-1).copy()


def support(seed: int, n: int, k: int) -> np.ndarray:
    """int64[k]: a uniform k-subset of [0, n), ascending."""
    out = np.empty(k, dtype=np.int64)
    if _load().l0gen_support(seed, n, k, _ptr(out)) != 0:
        raise ValueError(f"bad support arguments n={n} k={k}")
    return out


def values(seed: int, supp: np.ndarray, kind: int = VALUES_NORMAL) -> np.ndarray:
    """float64[k]: N(0,1) (kind 0) or uniform +-1 (kind 1) draws for supp."""
    supp = np.ascontiguousarray(supp, dtype=np.int64)
    out = np.empty(supp.size, dtype=np.float64)
    if _load().l0gen_values(seed, supp.size, _ptr(supp), kind, _ptr(out)) != 0:
        raise ValueError("bad value arguments")
    return out


def weights(seed: int, n: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """float64[n]: per-column weights of a column-scaled A, uniform on [lo, hi]."""
    out = np.empty(n, dtype=np.float64)
    if _load().l0gen_weights(seed, n, lo, hi, _ptr(out)) != 0:
        raise ValueError(f"bad weight arguments n={n} lo={lo} hi={hi}")
    return out


def banded_values(seed: int, supp: np.ndarray, band: float) -> np.ndarray:
    """float64[k]: N(0,1) nonzeros of which round(band * k), chosen uniformly
    (seeded), all equal one shared N(0,1) draw (the banded signals of the
    almost-dissociated experiments, Section 5)."""
    vals = values(seed, supp, VALUES_NORMAL)
    k = vals.size
    kb = int(round(float(band) * k))
    if kb:
        rng = np.random.Generator(np.random.PCG64(seed))
        pick = rng.choice(k, kb, replace=False)
        # the shared value: the N(0,1) draw of index 0 in a stream keyed apart
        vals[pick] = values(seed ^ 0x5EED5EED, np.zeros(1, dtype=np.int64))[0]
    return vals


def measure(n: int, m: int, d: int, col_idx: np.ndarray, supp: np.ndarray,
            vals: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """float64[m]: y = A x, each y_i summed from +0.0 over ascending columns;
    with weights w, column j of A holds w[j] and each term is fl(w[j] x_j)."""
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    supp = np.ascontiguousarray(supp, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float64)
        if w.shape != (n,):
            raise ValueError("weights must have n entries")
        wp = _ptr(w)
    y = np.empty(m, dtype=np.float64)
    if _load().l0gen_measure(n, m, d, _ptr(col_idx), supp.size, _ptr(supp), _ptr(vals), wp,
                             _ptr(y)) != 0:
        raise ValueError("bad measurement arguments")
    return y


@dataclass
class Instance:
    """One decoding problem: A (as col_idx), the true x and y = A x."""
    n: int
    m: int
    d: int
    k: int
    seed: int
    col_idx: np.ndarray   # int32[n*d]
    supp: np.ndarray      # int64[k], ascending
    vals: np.ndarray      # float64[k]
    y: np.ndarray         # float64[m]
    alpha: float
    kind: int = VALUES_NORMAL
    w: np.ndarray | None = None  # float64[n] column weights (column-scaled A), or None

    @property
    def x(self) -> np.ndarray:
        x = np.zeros(self.n, dtype=np.float64)
        x[self.supp] = self.vals
        return x


def default_alpha(d: int) -> float:
    """ceil(d/2), raised to 2 for d = 2 (alpha must lie in (1, d])."""
    return float(max(math.ceil(d / 2), 2))


def make_instance(seed: int, n: int, m: int, d: int, k: int, *, alpha: float | None = None,
                  kind: int = VALUES_NORMAL, scaled: bool = False) -> Instance:
    """Draw A, a k-sparse x and y = A x; alpha defaults to default_alpha(d).
    With scaled=True, A's columns carry weights uniform on [1/2, 3/2]."""
    col = columns(seed, n, m, d)
    supp = support(seed, n, k)
    vals = values(seed, supp, kind)
    w = weights(seed, n) if scaled else None
    y = measure(n, m, d, col, supp, vals, w)
    a = default_alpha(d) if alpha is None else float(alpha)
    return Instance(n, m, d, k, seed, col, supp, vals, y, a, kind, w)


# ---------------------------------------------------------------------------
# The five workloads.  m = round(delta*n), k = floor(rho*m); alpha = ceil(d/2).
# ---------------------------------------------------------------------------

def mk_m(n: int, delta: float) -> int:
    return int(round(delta * n))


def mk_k(m: int, rho: float) -> int:
    return int(math.floor(rho * m + 1e-9))


#: name -> (n, m, d, k) of the single-instance workloads.
SINGLE = {
    "small": (4096, 512, 7, 50),
    "n2^20": (1 << 20, mk_m(1 << 20, 0.1), 7, mk_k(mk_m(1 << 20, 0.1), 0.2)),
    "n2^24": (1 << 24, 16777, 7, mk_k(16777, 0.25)),
}


def single_workload(name: str, i: int = 0, kind: int = VALUES_NORMAL, scaled: bool = False) -> Instance:
    """Instance i of a single-instance workload ('small', 'n2^20', 'n2^24'),
    on a column-scaled A when scaled is set."""
    c = {"small": 0, "n2^20": 1, "n2^24": 2}[name]
    n, m, d, k = SINGLE[name]
    return make_instance(SEED + 1000 * c + i, n, m, d, k, kind=kind, scaled=scaled)


def sweep_params(count: int = 4096, seed: int = SEED + 3000):
    """Parameters of the batched phase-transition sweep.

    n = round(2^U), U ~ U[10, 18]; delta uniform over {0.01, 0.03, 0.1, 0.3};
    d uniform over {5, 7, 9}; rho ~ U[0.05, 0.5]; alpha = ceil(d/2).
    Returns a list of dicts with keys n, m, d, k, delta, rho, seed.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(10.0, 18.0, count)
    deltas = rng.choice(np.array([0.01, 0.03, 0.1, 0.3]), count)
    ds = rng.choice(np.array([5, 7, 9]), count)
    rhos = rng.uniform(0.05, 0.5, count)
    out = []
    for i in range(count):
        n = int(round(2.0 ** u[i]))
        m = max(mk_m(n, float(deltas[i])), int(ds[i]))
        k = mk_k(m, float(rhos[i]))
        out.append(dict(n=n, m=m, d=int(ds[i]), k=k, delta=float(deltas[i]),
                        rho=float(rhos[i]), seed=seed + 1 + i))
    return out


def serve_params(count: int = 2000, seed: int = SEED + 4000):
    """Request mix of the serving workload.

    n = round(2^U), U ~ U[12, 22]; delta uniform over {0.01, 0.1}; d = 7;
    k = floor(0.15 m); 10% of requests draw +-1 nonzeros.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(12.0, 22.0, count)
    deltas = rng.choice(np.array([0.01, 0.1]), count)
    pm1 = rng.uniform(0.0, 1.0, count) < 0.1
    out = []
    for i in range(count):
        n = int(round(2.0 ** u[i]))
        m = max(mk_m(n, float(deltas[i])), 7)
        out.append(dict(n=n, m=m, d=7, k=mk_k(m, 0.15), delta=float(deltas[i]),
                        kind=VALUES_PM1 if pm1[i] else VALUES_NORMAL, seed=seed + 1 + i))
    return out
