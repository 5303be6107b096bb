"""ORACLE — TEST INFRASTRUCTURE ONLY.

Brute-force sparsest solution of y = A x for tiny systems (n <= 20): the
problem Parallel-l0 and Serial-l0 aim at (Section 1, "recover the sparsest
solution"; Theorem 1.2).  Supports are enumerated by increasing size and each
is solved by least squares; the smallest size admitting an exact solution
whose entries are all nonzero gives the sparsest solutions.
"""
from __future__ import annotations

import itertools

import numpy as np


def dense_matrix(n: int, m: int, d: int, col_idx) -> np.ndarray:
    """The 0/1 adjacency matrix of Definition 2.2 (A_ij = 1 iff i in N(j))."""
    A = np.zeros((m, n), dtype=np.float64)
    cols = np.asarray(col_idx).reshape(n, d)
    for j in range(n):
        for i in cols[j]:
            A[i, j] = 1.0
    return A


def sparsest_solutions(A: np.ndarray, y: np.ndarray, *, rtol: float = 1e-9, max_size=None):
    """All sparsest x with A x = y (to rtol * max(1, ||y||_inf)).

    Returns (size, [x, ...]).  Size 0 means y = 0 and x = 0.
    """
    m, n = A.shape
    assert n <= 20, "brute force is only for tiny systems"
    scale = max(1.0, float(np.max(np.abs(y))) if y.size else 1.0)
    if np.max(np.abs(y), initial=0.0) <= rtol * scale:
        return 0, [np.zeros(n)]
    top = n if max_size is None else max_size
    for s in range(1, top + 1):
        found = []
        for S in itertools.combinations(range(n), s):
            AS = A[:, S]
            xs, *_ = np.linalg.lstsq(AS, y, rcond=None)
            if np.max(np.abs(AS @ xs - y)) <= rtol * scale and np.all(np.abs(xs) > rtol * scale):
                x = np.zeros(n)
                x[list(S)] = xs
                found.append(x)
        if found:
            return s, found
    return None, []


def is_dissociated(vals, *, rtol: float = 1e-12) -> bool:
    """Definition 1.1: all 2^k subset sums of the nonzeros are pairwise different.

    Sums closer than rtol * sum|vals| count as equal.  Intended for k <= 20.
    """
    vals = np.asarray(vals, dtype=np.float64)
    k = vals.size
    assert k <= 20
    sums = np.zeros(1)
    for v in vals:
        sums = np.concatenate([sums, sums + v])
    sums.sort()
    tol = rtol * max(1.0, float(np.sum(np.abs(vals))))
    return bool(np.all(np.diff(sums) > tol))
