"""ORACLE — TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``l0_oracle.c``, a plain FP64 CPU implementation of
Serial-l0 and Parallel-l0 (Algorithms 1 and 2 of Mendoza-Smith & Tanner,
"Expander l0-decoding"), plus :mod:`oracle.brute`, a brute-force sparsest
solver for tiny systems.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the GPU decoder
never calls it and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "l0_oracle.c")
_LIB = os.path.join(_HERE, "libl0oracle.so")
_LIB_OMP = os.path.join(_HERE, "libl0oracle_omp.so")

RULE_L0DEC = 0
RULE_MODE = 1
RULE_SHIFTED_L0DEC = 2  # Algorithm 3: one candidate per column per pass
RULE_SHIFTED_MODE = 3
TOL_RELATIVE, TOL_ABSOLUTE = 0, 1  # tau = tol * max_i |y_i|, or tau = tol
CONVERGED, STALLED, MAX_ITER = 0, 1, 2
OUTCOME_NAMES = {CONVERGED: "CONVERGED", STALLED: "STALLED", MAX_ITER: "MAX_ITER"}


def build(force: bool = True) -> str:
    """Compile ``libl0oracle.so`` (single-threaded) and ``libl0oracle_omp.so``
    (the same source with OpenMP) with gcc (-O2, no FP contraction, no
    fast-math)."""
    for lib, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                   "-std=c11", "-Wall", "-Wextra", "-Wno-unknown-pragmas", *extra, "-o", lib + ".tmp", _SRC,
                   "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(lib + ".tmp", lib)
    return _LIB


_lib = None
_lib_omp = None


def _load(threads: bool = False):
    """The single-threaded oracle library, or with threads=True its OpenMP
    build (same source, same results)."""
    global _lib, _lib_omp
    if threads:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP):
                build(force=False)
            _lib_omp = _declare(ctypes.CDLL(_LIB_OMP))
        return _lib_omp
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _declare(lib):
    """Argument and result types of the oracle's entry points."""
    P, I32, I64, F64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.orc_parallel_l0.argtypes = [I64, I32, I32, P, P, F64, I32, I32, F64, I32, P, P, P, P, P, P, P,
                                    P]
    lib.orc_parallel_l0.restype = ctypes.c_int
    lib.orc_serial_l0.argtypes = [I64, I32, I32, P, P, F64, I32, I32, F64, P, P, P, P, P]
    lib.orc_serial_l0.restype = ctypes.c_int
    lib.orc_residual.argtypes = [I64, I32, I32, P, P, P, P, P]
    lib.orc_residual.restype = None
    lib.orc_score_columns.argtypes = [I64, I32, P, P, F64, I32, I32, P, P, P]
    lib.orc_score_columns.restype = None
    lib.orc_score_columns_shifted.argtypes = [I64, I32, P, P, F64, I32, I32, I32, P, P]
    lib.orc_score_columns_shifted.restype = None
    lib.orc_literal_decrease.argtypes = [I32, I32, P, P, F64, F64]
    lib.orc_literal_decrease.restype = I32
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def parallel_l0(n, m, d, col_idx, y, alpha, *, max_iter=100, tol=1e-10, rule=RULE_L0DEC,
                x_init=None, w=None, tol_mode=TOL_RELATIVE, threads=False):
    """Run Parallel-l0 (rules L0DEC, MODE) or its shifted form (Algorithm 3;
    rules SHIFTED_L0DEC, SHIFTED_MODE), on a column-scaled A when column
    weights w are given (Section 4.3.3); returns dict(x, iters, outcome,
    trace, tsize, passes) where passes counts vote passes.  ValueError on
    invalid input, including a column that lists a row twice (A is binary
    with d ones per column, Definition 2.2).  threads=True runs the OpenMP
    build on all host cores (OMP_NUM_THREADS), bitwise the same result."""
    col_idx, y = _c(col_idx, np.int32), _c(y, np.float64)
    xi = None if x_init is None else _c(x_init, np.float64)
    wv = None if w is None else _c(w, np.float64)
    if wv is not None and wv.shape != (n,):
        raise ValueError("weights must have n entries")
    x = np.empty(n, dtype=np.float64)
    trace = np.zeros(max_iter + 1, dtype=np.int32)
    tsize = np.zeros(max(max_iter, 1), dtype=np.int64)
    iters, outcome, passes = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rc = _load(threads).orc_parallel_l0(n, m, d, _p(col_idx), _p(y), float(alpha), rule, max_iter,
                                 float(tol), int(tol_mode), _p(xi), _p(wv), _p(x), _p(trace), _p(tsize),
                                 ctypes.byref(iters), ctypes.byref(outcome), ctypes.byref(passes))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    it = iters.value
    return dict(x=x, iters=it, outcome=outcome.value, trace=trace[: it + 1].copy(),
                tsize=tsize[:it].copy(), passes=passes.value)


def serial_l0(n, m, d, col_idx, y, alpha, *, max_sweeps=100, tol=1e-10, rule=RULE_L0DEC):
    """Run Serial-l0; returns dict(x, updates, sweeps, outcome, final_nnz)."""
    col_idx, y = _c(col_idx, np.int32), _c(y, np.float64)
    x = np.empty(n, dtype=np.float64)
    upd, sw, oc, nnz = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rc = _load().orc_serial_l0(n, m, d, _p(col_idx), _p(y), float(alpha), rule, max_sweeps,
                               float(tol), _p(x), ctypes.byref(upd), ctypes.byref(sw),
                               ctypes.byref(oc), ctypes.byref(nnz))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return dict(x=x, updates=upd.value, sweeps=sw.value, outcome=oc.value, final_nnz=nnz.value)


def residual(n, m, d, col_idx, y, x, w=None):
    """r = y - A x with ascending-column sums from +0.0 (column weights w, if
    given, multiply each term once before it is added)."""
    col_idx, y, x = _c(col_idx, np.int32), _c(y, np.float64), _c(x, np.float64)
    wv = None if w is None else _c(w, np.float64)
    r = np.empty(m, dtype=np.float64)
    _load().orc_residual(n, m, d, _p(col_idx), _p(y), _p(x), _p(wv), _p(r))
    return r


def score_columns(rows, d, r, tau, a, rule=RULE_L0DEC):
    """Score the columns whose rows are rows[c*d:(c+1)*d] on residual r.

    Returns (sel uint8, omega float64, best int32) per column.
    """
    rows, r = _c(rows, np.int32), _c(r, np.float64)
    nc = rows.size // d
    sel = np.zeros(nc, dtype=np.uint8)
    omega = np.zeros(nc, dtype=np.float64)
    best = np.zeros(nc, dtype=np.int32)
    if nc:
        _load().orc_score_columns(nc, d, _p(rows), _p(r), float(tau), rule, int(a), _p(sel),
                                  _p(omega), _p(best))
    return sel, omega, best


def score_columns_shifted(rows, d, r, tau, a, t, rule=RULE_SHIFTED_L0DEC):
    """One shifted vote: each column tries only the value of r at its t-th
    neighbour.  Returns (sel uint8, omega float64) per column."""
    rows, r = _c(rows, np.int32), _c(r, np.float64)
    nc = rows.size // d
    sel = np.zeros(nc, dtype=np.uint8)
    omega = np.zeros(nc, dtype=np.float64)
    if nc:
        _load().orc_score_columns_shifted(nc, d, _p(rows), _p(r), float(tau), rule, int(a), int(t),
                                          _p(sel), _p(omega))
    return sel, omega


def literal_decrease(rows, r, omega, tau):
    """||r||_0 - ||r - omega a_j||_0 formed over the whole vector."""
    rows, r = _c(rows, np.int32), _c(r, np.float64)
    return int(_load().orc_literal_decrease(r.size, rows.size, _p(rows), _p(r), float(omega),
                                            float(tau)))


def zero_threshold(y, tol):
    """tau = tol * max_i |y_i| (the zero/equality threshold of a run)."""
    y = np.asarray(y, dtype=np.float64)
    return float(tol) * (float(np.max(np.abs(y))) if y.size else 0.0)
