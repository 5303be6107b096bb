"""The C-ABI library: it is built, loads, exports every entry point declared
in include/*.h, and rejects invalid arguments on the host before any device
work (these calls need no GPU)."""
import ctypes
import glob
import os
import re

import pytest

import paper_1508_01256_amd as l0

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w\s\*]*?\b(l0_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_builds_and_loads():
    assert os.path.exists(l0.LIB_PATH), "run __graft_entry__.build() first"
    L = l0.lib()
    assert l0.l0_version().startswith("l0decode")


def test_every_declared_symbol_is_exported():
    decl = declared_functions()
    assert set(decl) == set(l0.EXPORTED), decl
    L = ctypes.CDLL(l0.LIB_PATH)
    for name in decl:
        assert hasattr(L, name), name


def test_workspace_bytes_host_only():
    # at least the repacked index store (16-bit rows for m <= 65536, else
    # 32-bit) plus the per-row support lists (one int32 per edge)
    assert l0.l0_workspace_bytes(4096, 512, 7, 100) >= 4096 * 7 * (2 + 4)
    assert l0.l0_workspace_bytes(4096, 65536, 7, 100) >= 4096 * 7 * (2 + 4)
    assert l0.l0_workspace_bytes(4096, 65537, 7, 100) >= 4096 * 7 * (4 + 4)
    assert (l0.l0_workspace_bytes(4096, 65537, 7, 100) - l0.l0_workspace_bytes(4096, 65536, 7, 100)
            >= 4096 * 7 * 2)
    # invalid shapes give 0
    for args in [(0, 512, 7, 10), (4096, 0, 7, 10), (4096, 512, 1, 10), (4096, 512, 21, 10),
                 (10, 5, 7, 10), (4096, 512, 7, -1), (1 << 31, 512, 7, 10)]:
        assert l0.l0_workspace_bytes(*args) == 0, args


@pytest.mark.parametrize("bad", [
    dict(n=0), dict(m=0), dict(d=1), dict(d=21), dict(d=9, m=8), dict(alpha=1.0),
    dict(alpha=0.5), dict(alpha=7.5), dict(alpha=float("nan")), dict(max_iter=-1),
    dict(tol=-1e-3), dict(tol=float("inf")), dict(tol=float("nan")),
])
def test_argument_errors_are_rejected_before_device_work(bad):
    a = dict(n=4096, m=512, d=7, alpha=4.0, max_iter=10, tol=1e-10)
    a.update(bad)
    L = l0.lib()
    # null buffers are never dereferenced: the scalar checks come first
    st = L.l0_decode(None, a["n"], a["m"], a["d"], None, a["alpha"], a["max_iter"], a["tol"], None,
                     None, None)
    assert st == l0.L0_ERR_ARG
    st = L.l0_decode_ex(None, a["n"], a["m"], a["d"], None, a["alpha"], a["max_iter"], a["tol"],
                        None, None, None, None, 0, None)
    assert st == l0.L0_ERR_ARG


def test_bad_options_and_handles():
    L = l0.lib()
    o = l0.l0_opts(rule=5)
    st = L.l0_decode_ex(None, 4096, 512, 7, None, 4.0, 10, 1e-10, None, ctypes.byref(o), None, None,
                        0, None)
    assert st == l0.L0_ERR_ARG
    o = l0.l0_opts(tol_mode=3)
    assert L.l0_decode_ex(None, 4096, 512, 7, None, 4.0, 10, 1e-10, None, ctypes.byref(o), None,
                          None, 0, None) == l0.L0_ERR_ARG
    o = l0.l0_opts(reserved0=1)
    assert L.l0_decode_ex(None, 4096, 512, 7, None, 4.0, 10, 1e-10, None, ctypes.byref(o), None,
                          None, 0, None) == l0.L0_ERR_ARG
    assert L.l0_matrix_create(None, 4096, 512, 7, None, None) == l0.L0_ERR_ARG
    assert L.l0_solve(None, None, 4.0, 10, 1e-10, None, None, None, None, 0, None) == l0.L0_ERR_ARG
    assert L.l0_solve_workspace_bytes(None, 10) == 0
    assert L.l0_matrix_destroy(None) == l0.L0_OK


def test_status_strings():
    assert "CONVERGED" in l0.l0_status_string(0)
    assert l0.l0_status_string(l0.L0_DEV_BAD_INDEX) == "L0_DEV_BAD_INDEX"
    assert l0.l0_status_string(l0.L0_DEV_BAD_WEIGHT) == "L0_DEV_BAD_WEIGHT"


def _table(**over):
    p = dict(col_idx=None, n=4096, m=512, d=7, y=None, alpha=4.0, max_iter=10, reserved=0,
             tol=1e-10, x_out=None)
    p.update(over)
    arr = (l0.l0_problem * 2)()
    arr[0] = l0.l0_problem(None, 4096, 512, 7, None, 4.0, 10, 0, 1e-10, None)
    arr[1] = l0.l0_problem(p["col_idx"], p["n"], p["m"], p["d"], p["y"], p["alpha"], p["max_iter"],
                           p["reserved"], p["tol"], p["x_out"])
    return arr


@pytest.mark.parametrize("bad", [
    dict(n=0), dict(m=0), dict(d=1), dict(d=21), dict(d=9, m=8), dict(alpha=1.0), dict(alpha=7.5),
    dict(max_iter=-1), dict(tol=float("nan")), dict(reserved=1),
])
def test_batched_argument_errors(bad):
    L = l0.lib()
    t = _table(**bad)
    assert L.l0_batch_workspace_bytes(t, 2, None) == 0
    assert L.l0_decode_batched(t, 2, None, None, None, 0, None) == l0.L0_ERR_ARG
    o = l0.l0_batch_opts()
    assert L.l0_batch_autotune(t, 2, ctypes.byref(o), None, None, 0, None) == l0.L0_ERR_ARG


def test_batched_bad_options_and_counts():
    L = l0.lib()
    t = _table()
    # null device buffers are rejected before any device work
    assert L.l0_decode_batched(t, 2, None, None, None, 0, None) == l0.L0_ERR_ARG
    assert L.l0_decode_batched(None, 2, None, None, None, 0, None) == l0.L0_ERR_ARG
    assert L.l0_decode_batched(t, 0, None, None, None, 0, None) == l0.L0_ERR_ARG
    assert L.l0_batch_workspace_bytes(t, 0, None) == 0
    for o in [l0.l0_batch_opts(rule=4), l0.l0_batch_opts(tol_mode=2),
              l0.l0_batch_opts(block_threads=128), l0.l0_batch_opts(block_threads=1024),
              l0.l0_batch_opts(words_cap=-1), l0.l0_batch_opts(words_cap=63),
              l0.l0_batch_opts(words_cap=40000)]:
        assert L.l0_batch_workspace_bytes(t, 2, ctypes.byref(o)) == 0
        assert L.l0_decode_batched(t, 2, ctypes.byref(o), None, None, 0, None) == l0.L0_ERR_ARG
    # autotune needs an options record to write into
    assert L.l0_batch_autotune(t, 2, None, None, None, 0, None) == l0.L0_ERR_ARG


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes records have the C compiler's sizes and field offsets."""
    import subprocess
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "l0decode.h"\n'
        '#define F(T, f) printf(#T " " #f " %zu\\n", offsetof(T, f));\n'
        'int main(void) {\n'
        '  printf("l0_opts %zu\\n", sizeof(l0_opts));\n'
        '  printf("l0_problem %zu\\n", sizeof(l0_problem));\n'
        '  printf("l0_batch_opts %zu\\n", sizeof(l0_batch_opts));\n'
        '  printf("l0_result %zu\\n", sizeof(l0_result));\n'
        '  F(l0_problem, n) F(l0_problem, m) F(l0_problem, d) F(l0_problem, y) F(l0_problem, alpha)\n'
        '  F(l0_problem, max_iter) F(l0_problem, tol) F(l0_problem, x_out)\n'
        '  F(l0_opts, x_init) F(l0_opts, timeline) F(l0_opts, weights) F(l0_batch_opts, words_cap)\n'
        '  F(l0_problem, weights)\n'
        '  F(l0_batch_opts, timing)\n'
        '  printf("l0_server_opts %zu\\n", sizeof(l0_server_opts));\n'
        '  printf("l0_completion %zu\\n", sizeof(l0_completion));\n'
        '  F(l0_server_opts, batch) F(l0_completion, result) F(l0_completion, submit_s)\n'
        '  F(l0_completion, done_s)\n'
        '  F(l0_result, updates)\n'
        '  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", f"-I{os.path.join(ROOT, 'include')}",
                    "-I/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        parts = line.split()
        if len(parts) == 2:
            got[parts[0]] = int(parts[1])
        elif len(parts) == 3:
            got[parts[0] + "." + parts[1]] = int(parts[2])
    assert got["l0_opts"] == ctypes.sizeof(l0.l0_opts)
    assert got["l0_problem"] == ctypes.sizeof(l0.l0_problem)
    assert got["l0_batch_opts"] == ctypes.sizeof(l0.l0_batch_opts)
    assert got["l0_result"] == 24  # the binding's int64[3] result records
    assert got["l0_server_opts"] == ctypes.sizeof(l0.l0_server_opts)
    assert got["l0_completion"] == ctypes.sizeof(l0.l0_completion)
    assert got["l0_result"] == ctypes.sizeof(l0.l0_result)
    for name, cls in [("l0_problem", l0.l0_problem), ("l0_opts", l0.l0_opts),
                      ("l0_batch_opts", l0.l0_batch_opts), ("l0_server_opts", l0.l0_server_opts),
                      ("l0_completion", l0.l0_completion)]:
        for f, _ in cls._fields_:
            key = f"{name}.{f}"
            if key in got:
                assert got[key] == getattr(cls, f).offset, key
    assert got["l0_result.updates"] == 16
    assert got["l0_opts.weights"] == 48 and got["l0_problem.weights"] == 64


def test_server_argument_errors():
    L = l0.lib()
    h = ctypes.c_void_p()
    assert L.l0_server_create(None, ctypes.byref(h)) == l0.L0_ERR_ARG
    for o in [l0.l0_server_opts(0, 0, 0, l0.l0_batch_opts()),
              l0.l0_server_opts(1 << 20, -1, 0, l0.l0_batch_opts()),
              l0.l0_server_opts(1 << 20, 0, 5, l0.l0_batch_opts()),
              l0.l0_server_opts(1 << 20, 0, 0, l0.l0_batch_opts(rule=4)),
              l0.l0_server_opts(1 << 20, 0, 0, l0.l0_batch_opts(block_threads=1024)),
              l0.l0_server_opts(1 << 20, 0, 0, l0.l0_batch_opts(timing=1))]:
        assert L.l0_server_create(ctypes.byref(o), ctypes.byref(h)) == l0.L0_ERR_ARG
    o = l0.l0_server_opts(1 << 20, 0, 0, l0.l0_batch_opts())
    assert L.l0_server_create(ctypes.byref(o), None) == l0.L0_ERR_ARG
    assert L.l0_server_submit(None, None, 0) == l0.L0_ERR_ARG
    assert L.l0_server_poll(None, None, 0) == -l0.L0_ERR_ARG
    assert L.l0_server_drain(None) == l0.L0_ERR_ARG
    assert L.l0_server_outstanding(None) == 0
    assert L.l0_server_destroy(None) == l0.L0_OK
