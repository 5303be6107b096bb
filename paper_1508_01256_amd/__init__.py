"""Python binding of the l0decode C-ABI (include/l0decode.h).

Parallel-l0 expander decoding (Mendoza-Smith & Tanner, "Expander
l0-decoding", Algorithm 2) runs entirely in the HIP library
``libl0decode.so``; this module only marshals arguments.  PyTorch supplies
device memory and the current stream.  The same names as the C entry points
are exported (``l0_decode``, ``l0_decode_ex``, ``l0_solve`` ...), plus
:func:`decode` and :class:`Matrix` as conveniences over them.

Importing works without the library; the first call raises
:class:`LibraryMissing` if ``libl0decode.so`` has not been built (there is no
fallback path).
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libl0decode.so")

# status codes (returned)
L0_OK, L0_ERR_ARG, L0_ERR_OOM, L0_ERR_HIP, L0_ERR_WORKSPACE = 0, 1, 2, 3, 4
# outcomes (written on the device)
L0_CONVERGED, L0_STALLED, L0_MAX_ITER = 0, 1, 2
L0_DEV_BAD_INDEX, L0_DEV_NONFINITE_Y, L0_DEV_ABORTED, L0_DEV_BAD_WEIGHT = 16, 17, 19, 20
L0_DEV_REPEATED_ROW = 21
OUTCOME_NAMES = {0: "CONVERGED", 1: "STALLED", 2: "MAX_ITER", 16: "DEV_BAD_INDEX",
                 17: "DEV_NONFINITE_Y", 19: "DEV_ABORTED", 20: "DEV_BAD_WEIGHT",
                 21: "DEV_REPEATED_ROW"}
# rules and tolerance modes
L0_RULE_L0DEC, L0_RULE_MODE, L0_RULE_SHIFTED_L0DEC, L0_RULE_SHIFTED_MODE = 0, 1, 2, 3
L0_TOL_RELATIVE, L0_TOL_ABSOLUTE = 0, 1

#: every entry point declared in include/l0decode.h
EXPORTED = ("l0_version", "l0_status_string", "l0_decode", "l0_workspace_bytes", "l0_decode_ex",
            "l0_matrix_create", "l0_matrix_destroy", "l0_solve_workspace_bytes", "l0_solve", "l0_set_solve_admission",
            "l0_batch_workspace_bytes", "l0_decode_batched", "l0_batch_autotune",
            "l0_server_create", "l0_server_submit", "l0_server_poll", "l0_server_drain",
            "l0_server_outstanding", "l0_server_destroy", "l0_decode_noalloc",
            "l0_noalloc_workspace_bytes")


class LibraryMissing(RuntimeError):
    pass


class L0Error(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what} failed with status {status}")
        self.status = status


class l0_opts(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("tol_mode", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("reserved1", ctypes.c_int32),
                ("x_init", ctypes.c_void_p), ("trace", ctypes.c_void_p),
                ("tsize", ctypes.c_void_p), ("timeline", ctypes.c_void_p),
                ("weights", ctypes.c_void_p)]


class l0_problem(ctypes.Structure):
    _fields_ = [("col_idx", ctypes.c_void_p), ("n", ctypes.c_int64), ("m", ctypes.c_int32),
                ("d", ctypes.c_int32), ("y", ctypes.c_void_p), ("alpha", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tol", ctypes.c_double), ("x_out", ctypes.c_void_p),
                ("weights", ctypes.c_void_p)]


class l0_batch_opts(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("tol_mode", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("words_cap", ctypes.c_int32),
                ("timing", ctypes.c_void_p)]


class l0_result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outcome", ctypes.c_int32),
                ("final_nnz", ctypes.c_int32), ("support_size", ctypes.c_int32),
                ("updates", ctypes.c_int64)]


class l0_server_opts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_batch", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("batch", l0_batch_opts)]


class l0_completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("result", l0_result), ("submit_s", ctypes.c_double), ("launch_s", ctypes.c_double),
                ("done_s", ctypes.c_double)]


_lib = None


def lib():
    """The loaded ``libl0decode.so`` (ctypes), loading it on first use."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                                 "(or python -m paper_1508_01256_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, F64, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_size_t)
        L.l0_version.argtypes, L.l0_version.restype = [], ctypes.c_char_p
        L.l0_status_string.argtypes, L.l0_status_string.restype = [I32], ctypes.c_char_p
        L.l0_decode.argtypes = [P, I64, I32, I32, P, F64, I32, F64, P, P, P]
        L.l0_workspace_bytes.argtypes, L.l0_workspace_bytes.restype = [I64, I32, I32, I32], SZ
        L.l0_decode_ex.argtypes = [P, I64, I32, I32, P, F64, I32, F64, P, P, P, P, SZ, P]
        L.l0_matrix_create.argtypes = [P, I64, I32, I32, ctypes.POINTER(P), P]
        L.l0_matrix_destroy.argtypes = [P]
        L.l0_solve_workspace_bytes.argtypes, L.l0_solve_workspace_bytes.restype = [P, I32], SZ
        L.l0_solve.argtypes = [P, P, F64, I32, F64, P, P, P, P, SZ, P]
        L.l0_batch_workspace_bytes.argtypes = [P, I32, P]
        L.l0_batch_workspace_bytes.restype = SZ
        L.l0_decode_batched.argtypes = [P, I32, P, P, P, SZ, P]
        L.l0_batch_autotune.argtypes = [P, I32, P, P, P, SZ, P]
        L.l0_server_create.argtypes = [P, ctypes.POINTER(P)]
        L.l0_server_submit.argtypes = [P, P, I64]
        L.l0_server_poll.argtypes, L.l0_server_poll.restype = [P, P, I32], I32
        L.l0_server_drain.argtypes = [P]
        L.l0_server_outstanding.argtypes, L.l0_server_outstanding.restype = [P], I64
        L.l0_server_destroy.argtypes = [P]
        L.l0_set_solve_admission.argtypes = [I32, I32]
        L.l0_decode_noalloc.argtypes = [P, I64, I32, I32, P, F64, I32, F64, P, P, P]
        L.l0_noalloc_workspace_bytes.argtypes = [I64, I32, I32, I32]
        L.l0_noalloc_workspace_bytes.restype = SZ
        for f in ("l0_decode", "l0_decode_noalloc", "l0_decode_ex", "l0_matrix_create", "l0_matrix_destroy", "l0_solve",
                  "l0_set_solve_admission",
                  "l0_decode_batched", "l0_batch_autotune", "l0_server_create", "l0_server_submit",
                  "l0_server_drain", "l0_server_destroy"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(st, what):
    if st != L0_OK:
        raise L0Error(st, what)


# ---------------------------------------------------------------------------
# one-to-one wrappers of the C entry points (tensors in, status out)
# ---------------------------------------------------------------------------

def l0_version() -> str:
    return lib().l0_version().decode()


def l0_status_string(code: int) -> str:
    return lib().l0_status_string(code).decode()


def l0_decode(col_idx, n, m, d, y, alpha, max_iter, tol, x_out, iters_out) -> int:
    return lib().l0_decode(_ptr(col_idx), n, m, d, _ptr(y), float(alpha), max_iter, float(tol),
                           _ptr(x_out), _ptr(iters_out), _stream())


def l0_decode_noalloc(col_idx, n, m, d, y, alpha, max_iter, tol, x_out, iters_out) -> int:
    return lib().l0_decode_noalloc(_ptr(col_idx), n, m, d, _ptr(y), float(alpha), max_iter, float(tol),
                                   _ptr(x_out), _ptr(iters_out), _stream())


def l0_noalloc_workspace_bytes(n, m, d, max_iter) -> int:
    return lib().l0_noalloc_workspace_bytes(n, m, d, max_iter)


L0_NOALLOC_SCRATCH_BYTES = 128 << 20


def l0_workspace_bytes(n, m, d, max_iter) -> int:
    return lib().l0_workspace_bytes(n, m, d, max_iter)


def l0_set_solve_admission(max_members=0, window_us=0) -> int:
    """Cap the solve kernel's member workgroups and set the admission
    window (0 = defaults); results do not depend on either."""
    return lib().l0_set_solve_admission(int(max_members), int(window_us))


def _opts(rule, tol_mode, x_init, trace, tsize, timeline=None, weights=None):
    return l0_opts(rule, tol_mode, 0, 0, None if x_init is None else x_init.data_ptr(),
                   None if trace is None else trace.data_ptr(),
                   None if tsize is None else tsize.data_ptr(),
                   None if timeline is None else timeline.data_ptr(),
                   None if weights is None else weights.data_ptr())


def l0_decode_ex(col_idx, n, m, d, y, alpha, max_iter, tol, x_out, opts, res_out, workspace) -> int:
    return lib().l0_decode_ex(_ptr(col_idx), n, m, d, _ptr(y), float(alpha), max_iter, float(tol),
                              _ptr(x_out), None if opts is None else ctypes.byref(opts),
                              _ptr(res_out), _ptr(workspace),
                              0 if workspace is None else workspace.numel(), _stream())


def l0_matrix_create(col_idx, n, m, d):
    h = ctypes.c_void_p()
    st = lib().l0_matrix_create(_ptr(col_idx), n, m, d, ctypes.byref(h), _stream())
    return st, h


def l0_matrix_destroy(h) -> int:
    return lib().l0_matrix_destroy(h)


def l0_solve_workspace_bytes(h, max_iter) -> int:
    return lib().l0_solve_workspace_bytes(h, max_iter)


def l0_solve(h, y, alpha, max_iter, tol, x_out, opts, res_out, workspace) -> int:
    return lib().l0_solve(h, _ptr(y), float(alpha), max_iter, float(tol), _ptr(x_out),
                          None if opts is None else ctypes.byref(opts), _ptr(res_out),
                          _ptr(workspace), 0 if workspace is None else workspace.numel(), _stream())


def problem_table(problems):
    """A ctypes l0_problem array from dicts with keys col_idx, n, m, d, y,
    alpha, max_iter, tol, x_out and optionally weights (tensors for the
    buffers)."""
    arr = (l0_problem * len(problems))()
    for i, p in enumerate(problems):
        w = p.get("weights")
        arr[i] = l0_problem(p["col_idx"].data_ptr(), p["n"], p["m"], p["d"], p["y"].data_ptr(),
                            float(p["alpha"]), p["max_iter"], 0, float(p["tol"]),
                            p["x_out"].data_ptr(), None if w is None else w.data_ptr())
    return arr


def l0_batch_workspace_bytes(table, opts=None) -> int:
    return lib().l0_batch_workspace_bytes(table, len(table),
                                          None if opts is None else ctypes.byref(opts))


def l0_decode_batched(table, opts, results, workspace) -> int:
    return lib().l0_decode_batched(table, len(table), None if opts is None else ctypes.byref(opts),
                                   _ptr(results), _ptr(workspace),
                                   0 if workspace is None else workspace.numel(), _stream())


def l0_batch_autotune(table, opts, results, workspace) -> int:
    return lib().l0_batch_autotune(table, len(table), ctypes.byref(opts), _ptr(results),
                                   _ptr(workspace), 0 if workspace is None else workspace.numel(),
                                   _stream())


def l0_server_create(opts):
    h = ctypes.c_void_p()
    st = lib().l0_server_create(ctypes.byref(opts), ctypes.byref(h))
    return st, h


def l0_server_submit(h, problem, req_id) -> int:
    return lib().l0_server_submit(h, ctypes.byref(problem), int(req_id))


def l0_server_poll(h, out, cap) -> int:
    return lib().l0_server_poll(h, out, cap)


def l0_server_drain(h) -> int:
    return lib().l0_server_drain(h)


def l0_server_outstanding(h) -> int:
    return lib().l0_server_outstanding(h)


def l0_server_destroy(h) -> int:
    return lib().l0_server_destroy(h)


# ---------------------------------------------------------------------------
# conveniences
# ---------------------------------------------------------------------------

def _result_dict(res, trace, tsize, x):
    r = res.cpu()
    iters, outcome, final_nnz, support = (int(v) for v in r[:3].view(torch.int32)[:4].tolist())
    out = dict(x=x, iters=iters, outcome=outcome, final_nnz=final_nnz, support_size=support,
               updates=int(r[2].item()))
    if trace is not None and outcome < 16:
        out["trace"] = trace[: iters + 1].cpu()
    if tsize is not None and outcome < 16:
        out["tsize"] = tsize[:iters].cpu()
    return out


def new_result(device="cuda"):
    """A device buffer for one l0_result (24 bytes, as int64[3])."""
    return torch.zeros(3, dtype=torch.int64, device=device)


def decode(col_idx, y, n, m, d, alpha=None, *, max_iter=100, tol=1e-10, rule=L0_RULE_L0DEC,
           tol_mode=L0_TOL_RELATIVE, x_init=None, weights=None, want_trace=True):
    """Decode y = A x on the GPU via l0_decode_ex (column weights of a
    column-scaled A in `weights`, a device float64 tensor, or None); alpha
    defaults to max(ceil(d/2), 2), inside (1, d] for every d >= 2.  Returns a
    dict with x (device tensor), iters, outcome, final_nnz, support_size,
    updates, trace, tsize."""
    dev = y.device
    alpha = float(max(math.ceil(d / 2), 2)) if alpha is None else float(alpha)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    trace = torch.full((max_iter + 1,), -1, dtype=torch.int32, device=dev) if want_trace else None
    tsize = torch.zeros(max(max_iter, 1), dtype=torch.int64, device=dev) if want_trace else None
    res = new_result(dev)
    ws = torch.empty(l0_workspace_bytes(n, m, d, max_iter), dtype=torch.uint8, device=dev)
    o = _opts(rule, tol_mode, x_init, trace, tsize, weights=weights)
    _check(l0_decode_ex(col_idx, n, m, d, y, alpha, max_iter, tol, x, o, res, ws), "l0_decode_ex")
    torch.cuda.current_stream().synchronize()
    return _result_dict(res, trace, tsize, x)


def new_results(count, device="cuda"):
    """A device buffer for `count` l0_result records (as int64[count, 3])."""
    return torch.zeros((count, 3), dtype=torch.int64, device=device)


def results_list(results):
    """Host dicts (iters, outcome, final_nnz, support_size, updates) of a
    batched results buffer."""
    r = results.cpu()
    i32 = r[:, :2].contiguous().view(torch.int32).reshape(-1, 4).tolist()
    upd = r[:, 2].tolist()
    return [dict(iters=a, outcome=b, final_nnz=c, support_size=e, updates=u)
            for (a, b, c, e), u in zip(i32, upd)]


def decode_batched(problems, *, rule=L0_RULE_L0DEC, tol_mode=L0_TOL_RELATIVE, block_threads=0,
                   words_cap=0, autotune=False):
    """Decode many instances with l0_decode_batched.  `problems` are dicts as
    for problem_table; missing x_out buffers are allocated, alpha defaults to
    ceil(d/2), max_iter to 100, tol to 1e-10.  Returns (x list, result dicts)."""
    full = []
    for p in problems:
        q = dict(p)
        q.setdefault("alpha", float(max(math.ceil(q["d"] / 2), 2)))
        q.setdefault("max_iter", 100)
        q.setdefault("tol", 1e-10)
        if q.get("x_out") is None:
            q["x_out"] = torch.empty(q["n"], dtype=torch.float64, device=q["y"].device)
        full.append(q)
    table = problem_table(full)
    opts = l0_batch_opts(rule, tol_mode, block_threads, words_cap)
    dev = full[0]["y"].device
    results = new_results(len(full), dev)
    ws = torch.empty(l0_batch_workspace_bytes(table, None if autotune else opts), dtype=torch.uint8,
                     device=dev)
    if autotune:
        _check(l0_batch_autotune(table, opts, results, ws), "l0_batch_autotune")
    _check(l0_decode_batched(table, opts, results, ws), "l0_decode_batched")
    torch.cuda.current_stream().synchronize()
    return [q["x_out"] for q in full], results_list(results)


def _completion_dict(c):
    r = c.result
    return dict(id=c.id, status=c.status, iters=r.iters, outcome=r.outcome, final_nnz=r.final_nnz,
                support_size=r.support_size, updates=r.updates, submit_s=c.submit_s,
                launch_s=c.launch_s, done_s=c.done_s)


class Server:
    """A decoding server (l0_server_*): submit() queues a request, poll()
    makes progress and returns finished ones, drain() waits for all.  The
    request's tensors are kept referenced until its completion is returned."""

    def __init__(self, budget_bytes, *, max_batch=0, max_inflight=0, rule=L0_RULE_L0DEC,
                 tol_mode=L0_TOL_RELATIVE, block_threads=0, words_cap=0):
        self.opts = l0_server_opts(budget_bytes, max_batch, max_inflight,
                                   l0_batch_opts(rule, tol_mode, block_threads, words_cap, None))
        st, h = l0_server_create(self.opts)
        _check(st, "l0_server_create")
        self.handle = h
        self._keep = {}
        self._buf = (l0_completion * 256)()

    def submit(self, req_id, col_idx, y, n, m, d, x_out, alpha=None, max_iter=100, tol=1e-10,
               weights=None):
        alpha = float(max(math.ceil(d / 2), 2)) if alpha is None else float(alpha)
        prob = l0_problem(col_idx.data_ptr(), n, m, d, y.data_ptr(), alpha, max_iter, 0, float(tol),
                          x_out.data_ptr(), None if weights is None else weights.data_ptr())
        st = l0_server_submit(self.handle, prob, req_id)
        if st == L0_OK:
            self._keep[int(req_id)] = (col_idx, y, x_out, weights)
        return st

    def poll(self):
        out = []
        while True:
            k = l0_server_poll(self.handle, self._buf, len(self._buf))
            if k < 0:
                raise L0Error(-k, "l0_server_poll")
            for c in self._buf[:k]:
                self._keep.pop(int(c.id), None)
                out.append(_completion_dict(c))
            if k < len(self._buf):
                return out

    def drain(self):
        _check(l0_server_drain(self.handle), "l0_server_drain")
        return self.poll()

    def outstanding(self):
        return l0_server_outstanding(self.handle)

    def close(self):
        if self.handle:
            _check(l0_server_destroy(self.handle), "l0_server_destroy")
            self.handle = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Matrix:
    """A prepared matrix (l0_matrix_create); solve() runs l0_solve on it."""

    def __init__(self, col_idx, n, m, d):
        st, h = l0_matrix_create(col_idx, n, m, d)
        _check(st, "l0_matrix_create")
        self.handle, self.n, self.m, self.d = h, n, m, d
        self._ws = {}

    def workspace(self, max_iter):
        ws = self._ws.get(max_iter)
        if ws is None:
            nb = l0_solve_workspace_bytes(self.handle, max_iter)
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
            self._ws[max_iter] = ws
        return ws

    def solve_async(self, y, alpha, *, max_iter=100, tol=1e-10, rule=L0_RULE_L0DEC,
                    tol_mode=L0_TOL_RELATIVE, x=None, res=None, trace=None, tsize=None,
                    x_init=None, workspace=None, timeline=None, weights=None):
        """Enqueue one solve on the current stream; returns (x, res)."""
        x = torch.empty(self.n, dtype=torch.float64, device=y.device) if x is None else x
        res = new_result(y.device) if res is None else res
        ws = self.workspace(max_iter) if workspace is None else workspace
        o = _opts(rule, tol_mode, x_init, trace, tsize, timeline, weights)
        _check(l0_solve(self.handle, y, alpha, max_iter, tol, x, o, res, ws), "l0_solve")
        return x, res

    def solve(self, y, alpha, *, max_iter=100, tol=1e-10, rule=L0_RULE_L0DEC,
              tol_mode=L0_TOL_RELATIVE, x_init=None, weights=None, want_trace=True):
        trace = torch.full((max_iter + 1,), -1, dtype=torch.int32, device=y.device) if want_trace else None
        tsize = torch.zeros(max(max_iter, 1), dtype=torch.int64, device=y.device) if want_trace else None
        x, res = self.solve_async(y, alpha, max_iter=max_iter, tol=tol, rule=rule, tol_mode=tol_mode,
                                  trace=trace, tsize=tsize, x_init=x_init, weights=weights)
        torch.cuda.current_stream().synchronize()
        return _result_dict(res, trace, tsize, x)

    def close(self):
        if self.handle:
            _check(l0_matrix_destroy(self.handle), "l0_matrix_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
