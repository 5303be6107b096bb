#!/usr/bin/env python3
"""Benchmark: Parallel-l0 decoding of the n = 2^24 instance on one MI355X.

Workload: n = 2^24, m = 16777 (n/m ~ 10^3, residual held in LDS), d = 7,
k = floor(0.25 m) = 4194, nonzeros iid N(0,1) in FP64, alpha = ceil(d/2) = 4,
tol = 1e-10, max_iter = 100; A has d distinct uniform rows per column.
Inputs are seeded and synthetic and are resident in HBM before timing.

A step is one complete decode through the C-ABI (l0_decode_ex): repacking
the column-index store, then the persistent solve kernel (every vote,
residual update and ||r||_0 count until the loop stops).  `value` is decodes
per second.  The roofline object is for the dominant kernel, the persistent
solve kernel, timed with HIP events on the stream it runs on (torch's current
stream) over repeated l0_solve calls on the prepared matrix.  Its algorithmic
bytes per launch follow the method's per-pass figure: 8n (x_hat cleared) plus,
per vote pass, 4nd (the column-index stream at 4 bytes an index) + 16m (y
read, r written) plus (16 + 4d) per applied update.  The library stores
16-bit indices when m <= 65536, so the bytes it actually streams are fewer;
that figure is reported beside it ("stored_bytes_per_launch"), as are the
rocprofv3 counter bytes.  The CPU baseline is the FP64 oracle (one thread)
on one full decode of the same instance.
"""
from __future__ import annotations

import argparse
from concurrent.futures import ThreadPoolExecutor
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Parallel-ℓ0 solve time & HBM GB/s at n=2^24; batched solves/sec vs plain"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1508_01256_amd/csrc/l0_kernels.hip", "paper_1508_01256_amd/csrc/l0_internal.h",
                  "paper_1508_01256_amd/csrc/l0_filter.h", "paper_1508_01256_amd/csrc/l0_common.h"]
SIZES = ("n2^24", "n2^20")


def traffic_file(size: str) -> str:
    return os.path.join(ROOT, "profiles", f"solve_kernel_{size}_traffic.json")


def host_cpu():
    """(logical CPUs this process may use, CPU model name)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def oracle_threads():
    """Threads the OpenMP oracle build uses: OMP_NUM_THREADS when set, else
    every CPU this process may use."""
    cores, _ = host_cpu()
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", cores)))
    except ValueError:
        return cores


def oracle_pool_check(insts, results, xs, rule=0, alpha=None):
    """Run the single-threaded oracle on every instance (a thread pool over
    the instances: the oracle releases the GIL while it runs) and compare with
    the GPU's results: outcome, iterations and x_hat bitwise.  Returns
    (agree, checked, seconds, threads)."""
    import numpy as np

    import oracle
    threads = oracle_threads()

    def one(q):
        i = insts[q]
        o = oracle.parallel_l0(i.n, i.m, i.d, i.col_idx, i.y, i.alpha if alpha is None else alpha,
                               max_iter=100, tol=1e-10, rule=rule, w=i.w)
        r = results[q]
        return int(o["outcome"] == r["outcome"] and o["iters"] == r["iters"] and np.array_equal(o["x"], xs[q]))

    c0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as pool:
        agree = sum(pool.map(one, range(len(insts))))
    return agree, len(insts), time.perf_counter() - c0, threads


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(size="n2^24"):
    """HBM bytes per solve launch from the committed rocprofv3 counter runs,
    or None when the kernel source changed since they were taken."""
    try:
        with open(traffic_file(size)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def passes_of(iters, outcome):
    """Vote passes in a solve: one per iteration, plus the final one that
    finds no column to update when the run stalls."""
    return iters + (1 if outcome == 1 else 0)


def index_bytes(m):
    """Bytes per stored row index: the library keeps 16-bit rows when every
    row fits (m <= 65536), else 32-bit rows."""
    return 2 if m <= 65536 else 4


def word_mode(m):
    """Where the vote keeps the bucket words (as the library decides):
    1 = 32-bit in LDS, 2 = 16-bit folded in LDS, 3 = 8-bit folded in LDS,
    0 = 32-bit gathered from global memory."""
    lds = 144 * 1024
    if 4 * m <= lds:
        return 1
    if m <= 65536 and 2 * m <= lds:
        return 2
    return 3 if m <= lds else 0


def algorithmic_bytes(n, m, d, iters, outcome, tsizes, index_width=4):
    """Bytes of one solve launch by the method's per-pass figure (module doc):
    8n + passes * (index_width * n * d + 16m) + (16 + 4d) * sum |T|.  The
    method's figure takes 4-byte indices; index_width=index_bytes(m) gives
    the bytes of the store the library actually streams."""
    passes = passes_of(iters, outcome)
    b = 8 * n                                              # x_hat = 0
    b += passes * (index_width * n * d + 16 * m)            # index stream, y read + r write
    b += sum(int(t) for t in tsizes) * (16 + 4 * d)         # x_hat RMW + support-list appends
    return b, passes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=30, help="l0_solve launches timed for the roofline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--kind", choices=["normal", "pm1"], default="normal")
    ap.add_argument("--size", choices=SIZES, default="n2^24",
                    help="single: n=2^24, m=16777 (default) or n=2^20, m=104858")
    ap.add_argument("--no-sweep", action="store_true",
                    help="single: skip the batched-sweep leg reported in the line's detail")
    ap.add_argument("--workload", choices=["single", "sweep", "serve", "phase"], default="single",
                    help="single: one n=2^24 instance (default); sweep: 4096 phase-transition "
                         "instances through the batched decoder; serve: 2000 Poisson-arriving "
                         "requests through the decoding server; phase: 50%% recovery curves "
                         "rho*(delta) by the adaptive protocol of the paper's experiments")
    ap.add_argument("--phase-n", type=int, default=1 << 18, help="phase: problem size n")
    ap.add_argument("--phase-problems", type=int, default=10, help="phase: problems per (delta, rho)")
    ap.add_argument("--phase-curves", default="all", help="phase: comma-separated curve names, or all")
    ap.add_argument("--phase-check-every", type=int, default=400,
                    help="phase: every this many decoded instances is also run through the oracle")
    ap.add_argument("--phase-out", default="", help="phase: also write a markdown summary here")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--budget-gib", type=float, default=32.0, help="serve: server workspace budget")
    ap.add_argument("--serve-inflight", type=int, default=2, help="serve: server batches in flight (1..4)")
    ap.add_argument("--serve-loads", default="0.5,0.9,1.5", help="serve: loads as fractions of plain capacity")
    ap.add_argument("--sweep-count", type=int, default=4096)
    ap.add_argument("--autotune", action="store_true", help="sweep: pick the schedule with "
                    "l0_batch_autotune first")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 launches) to calibrate "
                         "rocprofv3 byte counters, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the decoder runs on "
              "one GPU", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1508_01256_amd as l0

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(args.calibrate_copy << 18, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_each_way": a.numel() * 4, "launches": 3}))
        return
    if args.workload == "sweep":
        return sweep(args)
    if args.workload == "serve":
        return serve(args)
    if args.workload == "phase":
        return phase(args)
    kind = gen.VALUES_NORMAL if args.kind == "normal" else gen.VALUES_PM1
    t0 = time.time()
    inst = gen.single_workload(args.size, 0, kind=kind)
    n, m, d, alpha, max_iter, tol = inst.n, inst.m, inst.d, inst.alpha, 100, 1e-10
    print(f"[bench] generated n={n} m={m} d={d} k={inst.k} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    col = torch.from_numpy(inst.col_idx).cuda()
    y = torch.from_numpy(inst.y).cuda()
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    res = l0.new_result()
    ws = torch.empty(l0.l0_workspace_bytes(n, m, d, max_iter), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        st = l0.l0_decode_ex(col, n, m, d, y, alpha, max_iter, tol, x, None, res, ws)
        if st != l0.L0_OK:
            raise RuntimeError(f"l0_decode_ex status {st}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    r = res.cpu()
    iters, outcome = (int(v) for v in r[:1].view(torch.int32).tolist())
    print(f"[bench] one-shot decode {ms_per_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f}), "
          f"iters={iters} outcome={l0.OUTCOME_NAMES[outcome]}", file=sys.stderr, flush=True)

    # dominant kernel: the persistent solve kernel on a prepared matrix
    A = l0.Matrix(col, n, m, d)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    A2 = l0.Matrix(col, n, m, d)
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - p0) * 1e3
    A2.close()
    trace = torch.full((max_iter + 1,), -1, dtype=torch.int32, device="cuda")
    tsize = torch.zeros(max_iter, dtype=torch.int64, device="cuda")
    xs, rs = A.solve_async(y, alpha, max_iter=max_iter, tol=tol, trace=trace, tsize=tsize)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.repeats)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.repeats)]
    for i in range(args.repeats):
        starts[i].record(stream)
        A.solve_async(y, alpha, max_iter=max_iter, tol=tol, x=xs, res=rs, trace=trace, tsize=tsize)
        ends[i].record(stream)
    torch.cuda.synchronize()
    solve_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    solve_avg = float(np.mean(solve_ms))
    rr = rs.cpu()
    s_iters, s_outcome = (int(v) for v in rr[:1].view(torch.int32).tolist())
    assert (s_iters, s_outcome) == (iters, outcome)
    assert torch.equal(xs, x), "prepared-matrix solve differs from the one-shot decode"
    # one more solve with the in-kernel phase timeline (device wall clock, 100 MHz)
    tl = torch.zeros(6 * max_iter + 16, dtype=torch.int64, device="cuda")
    A.solve_async(y, alpha, max_iter=max_iter, tol=tol, x=xs, res=rs, timeline=tl)
    torch.cuda.synchronize()
    tlv = tl.cpu().tolist()
    # entry 0: kernel start; 1..: grid barriers; 3*max_iter+7: every workgroup started
    bars = [tlv[0]] + [v for v in tlv[1:3 * max_iter + 7] if v > 0]
    phases_us = [round((bars[i + 1] - bars[i]) / 100.0, 1) for i in range(len(bars) - 1)]
    startup_us = round((tlv[3 * max_iter + 7] - tlv[0]) / 100.0, 1) if tlv[3 * max_iter + 7] else None
    sub = []
    for l in range(passes_of(iters, outcome)):
        b = 3 * max_iter + 8 + 3 * l
        if tlv[b + 2] > 0:
            prev = max(v for v in bars if v <= tlv[b])  # the barrier that opened this vote
            sub.append([round((tlv[b] - prev) / 100.0, 1), round((tlv[b + 1] - tlv[b]) / 100.0, 1),
                        round((tlv[b + 2] - tlv[b + 1]) / 100.0, 1)])
    print(f"[bench] phase timeline (us, between grid barriers): {phases_us}; all workgroups started "
          f"after {startup_us} us", file=sys.stderr, flush=True)
    print(f"[bench] vote sub-phases (us: stage, stream+filter, exact scoring): {sub}", file=sys.stderr,
          flush=True)
    ts = tsize[:iters].cpu().tolist()
    tr = trace[: iters + 1].cpu().tolist()
    bytes_launch, passes = algorithmic_bytes(n, m, d, iters, outcome, ts)
    stored_launch, _ = algorithmic_bytes(n, m, d, iters, outcome, ts, index_width=index_bytes(m))
    achieved = bytes_launch / (solve_avg * 1e-3) / 1e9
    stored_gbs = stored_launch / (solve_avg * 1e-3) / 1e9
    vote_bytes = index_bytes(m) * n * d
    print(f"[bench] solve kernel avg {solve_avg:.3f} ms (min {min(solve_ms):.3f}) over {args.repeats}; "
          f"passes={passes} trace={tr} tsize={ts}; {achieved:.0f} GB/s algorithmic "
          f"({stored_gbs:.0f} GB/s of the {8 * index_bytes(m)}-bit store actually streamed); "
          f"prep {prep_ms:.2f} ms", file=sys.stderr, flush=True)
    A.close()

    traffic = measured_traffic(args.size)
    kname = f"l0::solve_kernel<{d},{word_mode(m)}>"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "bytes_per_launch": bytes_launch,
                "avg_launch_ms": round(solve_avg, 4), "stored_bytes_per_launch": stored_launch,
                "stored_gbs": round(stored_gbs, 1)}
    if traffic:
        # the bytes the counters saw per launch, over the same launch time
        roofline["counter_gbs"] = round(traffic / (solve_avg * 1e-3) / 1e9, 1)
        roofline["counter_frac"] = round(traffic / (solve_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    if stored_launch < bytes_launch:
        roofline["note"] = ("frac counts the method's 4-byte indices; the library streams "
                            f"{8 * index_bytes(m)}-bit ones (stored_gbs), so frac can pass 1; "
                            "counter_frac is the memory system's fraction")
    gx = xs.cpu().numpy()
    del xs, rs, x, res, ws, trace, tsize, tl

    cpu = None
    if not args.no_cpu:
        import oracle
        cores, model = host_cpu()
        c0 = time.perf_counter()
        o1 = oracle.parallel_l0(n, m, d, inst.col_idx, inst.y, alpha, max_iter=max_iter, tol=tol)
        t1 = time.perf_counter() - c0
        threads = oracle_threads()
        c0 = time.perf_counter()
        on = oracle.parallel_l0(n, m, d, inst.col_idx, inst.y, alpha, max_iter=max_iter, tol=tol, threads=True)
        tn = time.perf_counter() - c0
        ok1 = o1["iters"] == iters and np.array_equal(o1["x"], gx)
        okn = on["iters"] == iters and np.array_equal(on["x"], gx)
        cpu = {"value": round(1.0 / tn, 5), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"1 full decode of the same {args.size} instance with the oracle's OpenMP build "
                         f"({tn:.2f} s on {threads} threads of {cores} CPUs, {model}); the plain "
                         f"single-threaded build {t1:.2f} s ({1.0 / t1:.4f} solves/s); gcc -O2; parity "
                         f"with GPU: {'bitwise' if ok1 and okn else 'MISMATCH'}",
               "single_thread_value": round(1.0 / t1, 5)}
        print(f"[bench] oracle {t1:.2f} s/solve on 1 thread, {tn:.2f} s on {threads}, parity "
              f"{'ok' if ok1 and okn else 'MISMATCH'}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_per_step, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Parallel-l0 single instance n={args.size[1:]} m={m} d={d} k={inst.k} "
                               f"alpha={alpha:g} tol={tol:g} max_iter={max_iter} "
                               f"{'N(0,1)' if kind == 0 else 'uniform +-1'} nonzeros, seed {inst.seed}",
                   "n": n, "m": m, "d": d, "k": inst.k, "alpha": alpha, "step": "l0_decode_ex (repack + solve)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {"iters": iters, "outcome": l0.OUTCOME_NAMES[outcome], "trace": tr, "tsize": ts,
                   "vote_passes": passes, "solve_prepared_ms": round(solve_avg, 4),
                   "solve_prepared_min_ms": round(min(solve_ms), 4),
                   "per_vote_pass_us": round(solve_avg * 1e3 / max(passes, 1), 2),
                   "vote_bytes_per_pass": vote_bytes, "prepare_ms": round(prep_ms, 3),
                   "solves_per_s_prepared": round(1e3 / solve_avg, 3),
                   "phase_us": phases_us, "startup_us": startup_us},
    }
    if not args.no_sweep:
        # the metric's second half: the batched decoder against the plain
        # one-launch-per-instance loop on the 4096-instance sweep
        out["detail"]["batched_sweep"] = run_sweep(args.sweep_count, steps=5, warmup=1,
                                                   check=not args.no_cpu)["summary"]
    print(json.dumps(out), flush=True)


def release_device():
    """Free what torch's caching allocator holds before the interpreter
    exits (nothing of the device is left for static destructors to free)."""
    import gc

    import torch
    if not torch.cuda.is_initialized():
        return
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def solve_bytes(n, m, d, iters, outcome, tsizes):
    """Algorithmic bytes of one decode with 32-bit indices: 8n (x_hat zeroed)
    plus, per vote pass, 4nd + 16m + (16 + 4d)|T|."""
    passes = passes_of(iters, outcome)
    return 8 * n + passes * (4 * n * d + 16 * m) + sum((16 + 4 * d) * t for t in tsizes)


def run_sweep(count, steps, warmup, check=True, autotune=False, schedule=(512, 32768)):
    """The batched phase-transition sweep: all instances in one
    l0_decode_batched call per step (timed over `steps`), against a plain
    loop of one l0_decode_ex per instance on one stream; per-(delta, rho)
    cell success; with `check`, every instance against the oracle.  Returns
    dict(summary=..., ms_per_step, bytes_total, schedule, cpu)."""
    import numpy as np
    import torch

    import gen
    import paper_1508_01256_amd as l0

    params = gen.sweep_params(4096)[:count]
    t0 = time.time()
    insts = [gen.make_instance(p["seed"], p["n"], p["m"], p["d"], p["k"]) for p in params]
    dev = "cuda"
    probs = [dict(col_idx=torch.from_numpy(i.col_idx).to(dev), n=i.n, m=i.m, d=i.d,
                  y=torch.from_numpy(i.y).to(dev), alpha=i.alpha, max_iter=100, tol=1e-10,
                  x_out=torch.empty(i.n, dtype=torch.float64, device=dev)) for i in insts]
    torch.cuda.synchronize()
    print(f"[bench] generated and uploaded {count} sweep instances in {time.time() - t0:.1f}s "
          f"(index bytes {sum(4 * i.n * i.d for i in insts) / 1e9:.2f} GB)", file=sys.stderr, flush=True)
    table = l0.problem_table(probs)
    opts = l0.l0_batch_opts(0, 0, *schedule)
    results = l0.new_results(count, dev)
    if autotune:
        ws = torch.empty(l0.l0_batch_workspace_bytes(table, None), dtype=torch.uint8, device=dev)
        st = l0.l0_batch_autotune(table, opts, results, ws)
        assert st == l0.L0_OK, st
        print(f"[bench] autotuned schedule: {opts.block_threads} threads, {opts.words_cap} words",
              file=sys.stderr, flush=True)
    else:
        ws = torch.empty(l0.l0_batch_workspace_bytes(table, opts), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        st = l0.l0_decode_batched(table, opts, results, ws)
        if st != l0.L0_OK:
            raise RuntimeError(f"l0_decode_batched status {st}")

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = e0.elapsed_time(e1) / steps
    rl = l0.results_list(results)
    xs = [p["x_out"].cpu().numpy() for p in probs]

    # per-instance record of the timed configuration (one more step)
    tim = torch.zeros((count, 8), dtype=torch.int64, device=dev)
    topts = l0.l0_batch_opts(opts.rule, opts.tol_mode, opts.block_threads, opts.words_cap, tim.data_ptr())
    assert l0.l0_decode_batched(table, topts, results, ws) == l0.L0_OK
    torch.cuda.synchronize()
    T = tim.cpu().numpy().astype(np.float64) / 100.0
    span_us = T[:, 1].max() - T[:, 0].min()
    phase_ms = {k: round(float(T[:, c].sum()) / 1e3, 1) for k, c in
                (("setup", 2), ("vote", 3), ("score", 4), ("residual", 5))}
    busy = float((T[:, 1] - T[:, 0]).sum())

    # plain path: one l0_decode_ex per instance on one stream
    mx = max(l0.l0_workspace_bytes(i.n, i.m, i.d, 100) for i in insts)
    ws1 = torch.empty(mx, dtype=torch.uint8, device=dev)
    r1 = l0.new_result(dev)
    xp = [torch.empty(i.n, dtype=torch.float64, device=dev) for i in insts]
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for p, x in zip(probs, xp):
        st = l0.l0_decode_ex(p["col_idx"], p["n"], p["m"], p["d"], p["y"], p["alpha"], 100, 1e-10,
                             x, None, r1, ws1)
        assert st == l0.L0_OK
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - p0
    same = all(torch.equal(a, b["x_out"]) for a, b in zip(xp, probs))
    del xp, ws1, ws, probs, tim

    # success (||x_hat - x||_inf <= 1e-12 ||x||_inf; k = 0: x_hat = 0) per (delta, rho-bin) cell
    def success(i, x):
        if i.k == 0:
            return not np.any(x)
        xt = i.x
        return float(np.max(np.abs(x - xt))) <= 1e-12 * float(np.max(np.abs(xt)))

    succ = [success(i, x) and r["outcome"] == l0.L0_CONVERGED for i, x, r in zip(insts, xs, rl)]
    cells = {}
    for p, ok in zip(params, succ):
        key = f"delta={p['delta']:g} rho=[{int(p['rho'] / 0.05) * 0.05:.2f},{int(p['rho'] / 0.05) * 0.05 + 0.05:.2f})"
        a, b = cells.get(key, (0, 0))
        cells[key] = (a + int(ok), b + 1)

    cpu = None
    agree = checked = None
    if check:
        # every instance through the oracle: the per-cell success counts are
        # then the oracle's too (an instance agrees only if outcome,
        # iterations and x_hat are bitwise equal)
        agree, checked, cdt, threads = oracle_pool_check(insts, rl, xs)
        cores, model = host_cpu()
        cpu = {"value": round(checked / cdt, 3), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"all {checked} instances, single-threaded oracle on a pool of {threads} threads "
                         f"({cores} CPUs, {model}), {cdt:.1f} s; {agree}/{checked} bitwise equal to the "
                         "batched GPU results"}
    # algorithmic bytes: per instance, vote passes from the outcome; the |T| term is linear, so
    # the total update count gives it exactly
    bytes_total = 0
    for i, r in zip(insts, rl):
        it, oc = r["iters"], r["outcome"]
        bytes_total += solve_bytes(i.n, i.m, i.d, it, oc, [r["updates"]] if it else [])
    achieved = bytes_total / (ms_per_step * 1e-3) / 1e9
    print(f"[bench] batched {ms_per_step:.2f} ms per sweep ({count / ms_per_step * 1e3:.0f} solves/s); "
          f"plain loop {plain_s * 1e3:.1f} ms ({count / plain_s:.0f} solves/s), same x: {same}; "
          f"span {span_us / 1e3:.2f} ms, workgroup-busy {busy / 1e3:.0f} ms, phases {phase_ms}; "
          f"oracle agreement {agree}/{checked}", file=sys.stderr, flush=True)
    for key in sorted(cells):
        a, b = cells[key]
        print(f"[bench]   {key}: {a}/{b} recovered", file=sys.stderr)
    summary = {"instances": count, "ms_per_sweep": round(ms_per_step, 3),
               "solves_per_s": round(count / ms_per_step * 1e3, 1),
               "plain_loop_solves_per_s": round(count / plain_s, 1),
               "speedup_vs_plain": round(plain_s * 1e3 / ms_per_step, 2),
               "plain_results_identical": same, "gbs_method_bytes": round(achieved, 1),
               "frac": round(achieved / HBM_PEAK_GBS, 4),
               "schedule": {"block_threads": opts.block_threads, "words_cap": opts.words_cap},
               "oracle_agree": agree, "oracle_checked": checked, "recovered": int(sum(succ))}
    return dict(summary=summary, ms_per_step=ms_per_step, bytes_total=bytes_total, achieved=achieved,
                cpu=cpu, cells=cells, span_ms=span_us / 1e3, busy_ms=busy / 1e3, phase_ms=phase_ms,
                outcomes={l0.OUTCOME_NAMES[k]: int(sum(r["outcome"] == k for r in rl)) for k in (0, 1, 2)})


def sweep(args):
    """The batched phase-transition sweep as a bench line of its own."""
    count = args.sweep_count
    r = run_sweep(count, args.steps, args.warmup, check=not args.no_cpu, autotune=args.autotune)
    sm = r["summary"]
    out = {
        "metric": "batched Parallel-l0 solves/s on the phase-transition sweep vs a plain loop",
        "value": sm["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sm["ms_per_sweep"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{count} instances, n=round(2^U) U~U[10,18], delta in "
                               "{0.01,0.03,0.1,0.3}, d in {5,7,9}, rho~U[0.05,0.5], alpha=ceil(d/2), "
                               "max_iter=100, tol=1e-10, N(0,1) nonzeros",
                   "schedule": sm["schedule"]},
        "roofline": {"bound": "hbm", "achieved": round(r["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["achieved"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "l0::batch_kernel (all launches of one sweep)",
                     "bytes_per_launch": r["bytes_total"]},
        "cpu_baseline": r["cpu"],
        "detail": {**{k: v for k, v in sm.items() if k not in ("schedule",)},
                   "span_ms": round(r["span_ms"], 3), "workgroup_busy_ms": round(r["busy_ms"], 1),
                   "phase_ms": r["phase_ms"], "outcomes": r["outcomes"],
                   "cells": {k: f"{a}/{b}" for k, (a, b) in sorted(r["cells"].items())}},
    }
    print(json.dumps(out), flush=True)


def serve(args):
    """Serving mix under Poisson arrivals: the decoding server (continuous
    batching under an HBM budget) against the plain path (one l0_decode_ex
    per request, in arrival order), at 0.5, 0.9 and 1.5 times the plain
    path's measured capacity."""
    import numpy as np
    import torch

    import gen
    import paper_1508_01256_amd as l0

    params = gen.serve_params(args.serve_count)
    t0 = time.time()
    insts = [gen.make_instance(p["seed"], p["n"], p["m"], p["d"], p["k"], kind=p["kind"]) for p in params]
    dev = "cuda"
    reqs = [dict(col=torch.from_numpy(i.col_idx).to(dev), y=torch.from_numpy(i.y).to(dev),
                 x=torch.empty(i.n, dtype=torch.float64, device=dev), n=i.n, m=i.m, d=i.d, alpha=i.alpha)
            for i in insts]
    del insts
    torch.cuda.synchronize()
    count = len(reqs)
    print(f"[bench] generated and uploaded {count} requests in {time.time() - t0:.1f}s "
          f"(index bytes {sum(4 * r['n'] * r['d'] for r in reqs) / 1e9:.1f} GB)", file=sys.stderr, flush=True)

    # plain path: workspace for the largest request, results as the reference
    ws = torch.empty(max(l0.l0_workspace_bytes(r["n"], r["m"], r["d"], 100) for r in reqs), dtype=torch.uint8,
                     device=dev)
    res1 = l0.new_result(dev)

    def plain_one(r, x):
        st = l0.l0_decode_ex(r["col"], r["n"], r["m"], r["d"], r["y"], r["alpha"], 100, 1e-10, x, None, res1, ws)
        assert st == l0.L0_OK, st

    for r in reqs[:20]:
        plain_one(r, r["x"])
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for r in reqs:
        plain_one(r, r["x"])
    torch.cuda.synchronize()
    capacity = count / (time.perf_counter() - c0)
    ref = [r["x"].clone() for r in reqs]
    print(f"[bench] plain path capacity {capacity:.0f} requests/s", file=sys.stderr, flush=True)

    def pct(v, q):
        return float(np.percentile(np.asarray(v), q))

    rng = np.random.Generator(np.random.PCG64(gen.SEED + 4500))
    runs = []
    for factor in [float(v) for v in args.serve_loads.split(",")]:
        lam = factor * capacity
        arrivals = np.cumsum(rng.exponential(1.0 / lam, count))
        # plain path: FIFO, one request at a time, starting when it has arrived
        lat_plain = []
        start = time.perf_counter()
        for r, a in zip(reqs, arrivals):
            while time.perf_counter() - start < a:
                pass
            plain_one(r, r["x"])
            torch.cuda.synchronize()
            lat_plain.append(time.perf_counter() - start - a)
        span_plain = time.perf_counter() - start
        # server: submit at arrival, poll continuously
        for r in reqs:
            r["x"].zero_()
        torch.cuda.synchronize()
        srv = l0.Server(int(args.budget_gib * (1 << 30)), max_inflight=args.serve_inflight)
        lat_srv = [None] * count
        nsub = 0
        start = time.perf_counter()
        batches = set()
        while True:
            now = time.perf_counter() - start
            while nsub < count and arrivals[nsub] <= now:
                r = reqs[nsub]
                st = srv.submit(nsub, r["col"], r["y"], r["n"], r["m"], r["d"], r["x"], r["alpha"])
                assert st == l0.L0_OK, st
                nsub += 1
            for c in srv.poll():
                assert c["status"] == l0.L0_OK
                lat_srv[c["id"]] = time.perf_counter() - start - arrivals[c["id"]]
                batches.add(c["launch_s"])
            if nsub == count and srv.outstanding() == 0:
                break
        span_srv = time.perf_counter() - start
        srv.close()
        same = all(torch.equal(r["x"], x) for r, x in zip(reqs, ref))
        run = {"load": factor, "lambda_per_s": round(lam, 1),
               "server": {"p50_ms": round(pct(lat_srv, 50) * 1e3, 3), "p99_ms": round(pct(lat_srv, 99) * 1e3, 3),
                          "solves_per_s": round(count / span_srv, 1), "batches": len(batches)},
               "plain": {"p50_ms": round(pct(lat_plain, 50) * 1e3, 3), "p99_ms": round(pct(lat_plain, 99) * 1e3, 3),
                         "solves_per_s": round(count / span_plain, 1)},
               "results_equal_solo": same}
        runs.append(run)
        print(f"[bench] load {factor}: {json.dumps(run)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        import oracle
        small = [q for q in range(count) if params[q]["n"] <= (1 << 16)][:40]
        c0 = time.perf_counter()
        agree = 0
        for q in small:
            i = gen.make_instance(params[q]["seed"], params[q]["n"], params[q]["m"], 7, params[q]["k"],
                                  kind=params[q]["kind"])
            o = oracle.parallel_l0(i.n, i.m, i.d, i.col_idx, i.y, i.alpha, max_iter=100, tol=1e-10)
            agree += int(np.array_equal(o["x"], ref[q].cpu().numpy()))
        cdt = time.perf_counter() - c0
        cpu = {"value": round(len(small) / cdt, 2), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(small)} requests with n <= 2^16 (generation included), {cdt:.1f} s single "
                         f"thread; {agree}/{len(small)} bitwise equal to the GPU results"}
    top = runs[-1]
    out = {
        "metric": "serving: p50/p99 arrival-to-result latency and solves/s under Poisson arrivals",
        "value": top["server"]["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{count} requests, n=round(2^U) U~U[12,22], delta in {{0.01,0.1}}, d=7, "
                               "k=floor(0.15m), 10% +-1 nonzeros, Poisson arrivals at 0.5/0.9/1.5 x the plain "
                               "path's capacity", "budget_gib": args.budget_gib, "max_inflight": args.serve_inflight},
        "roofline": None,
        "cpu_baseline": cpu,
        "detail": {"plain_capacity_per_s": round(capacity, 1), "runs": runs},
    }
    print(json.dumps(out), flush=True)


# name -> (d, alpha, rule, values, scaled columns, band): the paper's protocol at its experimental
# alpha = 2 with Algorithm 2's score; the frequency rule at alpha = 2 and at alpha = d/2 (the
# latter is parallel-LDDSR as Section 4.3.2 defines it, the frequency score with epsilon = 1/4,
# i.e. alpha = (1 - 2 epsilon) d); the workloads' alpha = ceil(d/2); the shifted rule; banded
# signals (Section 5.6); the odd degrees 5 to 19 (Section 5.7); and +-1 signals on unit and on
# column-scaled A (Section 4.3.3).
PHASE_CURVES = {
    "l0dec-a2": (7, 2.0, "L0DEC", "normal", False, 0.0),
    "mode-a2": (7, 2.0, "MODE", "normal", False, 0.0),
    "lddsr-ad2": (7, 3.5, "MODE", "normal", False, 0.0),
    "l0dec-a4": (7, 4.0, "L0DEC", "normal", False, 0.0),
    "shifted-a2": (7, 2.0, "SHIFTED_L0DEC", "normal", False, 0.0),
    "band0.5-a2": (7, 2.0, "L0DEC", "normal", False, 0.5),
    "band0.9-a2": (7, 2.0, "L0DEC", "normal", False, 0.9),
    "d5-a2": (5, 2.0, "L0DEC", "normal", False, 0.0),
    "d9-a2": (9, 2.0, "L0DEC", "normal", False, 0.0),
    "d11-a2": (11, 2.0, "L0DEC", "normal", False, 0.0),
    "d13-a2": (13, 2.0, "L0DEC", "normal", False, 0.0),
    "d15-a2": (15, 2.0, "L0DEC", "normal", False, 0.0),
    "d17-a2": (17, 2.0, "L0DEC", "normal", False, 0.0),
    "d19-a2": (19, 2.0, "L0DEC", "normal", False, 0.0),
    "pm1-a2": (7, 2.0, "L0DEC", "pm1", False, 0.0),
    "pm1-scaled-a2": (7, 2.0, "L0DEC", "pm1", True, 0.0),
}


def phase_deltas():
    """The delta grid of the paper's phase-transition protocol (Section 5.1):
    0.02 p for p = 1..4, then 0.1 + 89 (p - 1) / 1900 for p = 1..20."""
    return [0.02 * p for p in range(1, 5)] + [0.1 + 89.0 * (p - 1) / 1900.0 for p in range(1, 21)]


def logistic_50(rhos, succ, total):
    """50% point of a logistic fit p(rho) = 1 / (1 + exp((rho - rho_star) / s))
    to success counts (binomial likelihood; a weak prior on log s keeps the
    fit finite when successes and failures separate perfectly)."""
    import numpy as np
    from scipy.optimize import minimize

    r = np.asarray(rhos, float)
    k = np.asarray(succ, float)
    t = np.asarray(total, float)
    if k.sum() == 0:
        return None
    if k.sum() == t.sum():
        return float(r.max())

    def nll(th):
        z = (r - th[0]) / np.exp(th[1])
        # log p = -log(1 + e^z), log(1 - p) = z - log(1 + e^z)
        lp = -np.logaddexp(0.0, z)
        lq = z - np.logaddexp(0.0, z)
        return -(k * lp + (t - k) * lq).sum() + 1e-3 * (th[1] - np.log(0.01)) ** 2

    mid = float(np.sum(r * k) / np.sum(k))
    best = min((minimize(nll, np.array([x0, np.log(0.01)]), method="Nelder-Mead",
                         options={"xatol": 1e-7, "fatol": 1e-10, "maxiter": 4000})
                for x0 in (mid, float(r[k > 0].max()))), key=lambda o: o.fun)
    return float(best.x[0])


def phase_protocol(curve, n, problems, decode, log, check_every=0, start=0):
    """Run the adaptive protocol for one curve: for each delta start at
    rho = 0.01 with `problems` instances; while at least one is recovered,
    raise rho by 0.01.  decode(insts, alpha, rule, keep) returns per instance
    (outcome, iters, relative error ||x_hat - x||_inf / ||x||_inf, x_hat or
    None), x_hat on the host where keep is set.  Every check_every-th decoded
    instance (counting from `start` over all curves) is kept.  Returns per
    delta the (rho, successes) points, the kept records and the count of
    instances decoded."""
    import numpy as np

    import gen

    d, alpha, rule, kind, scaled, band = PHASE_CURVES[curve]
    deltas = phase_deltas()
    mats = {}

    def matrix(di, q):
        key = (di, q)
        if key not in mats:
            m = int(round(deltas[di] * n))
            seed = gen.SEED + 5000 + 100000 * d + 100 * di + q
            mats[key] = (m, seed, gen.columns(seed, n, m, d), gen.weights(seed, n) if scaled else None)
        return mats[key]

    points = {di: [] for di in range(len(deltas))}
    active = list(range(len(deltas)))
    step = 0
    records = []
    len_done = 0
    while active:
        rho = round(0.01 * (step + 1), 2)
        def draw(di, q):
            m, seed, col, w = matrix(di, q)
            k = min(int(np.floor(rho * m + 1e-9)), n)
            sseed = seed * 1009 + step
            supp = gen.support(sseed, n, k)
            if kind == "pm1":
                vals = gen.values(sseed, supp, gen.VALUES_PM1)
            else:
                vals = gen.banded_values(sseed, supp, band)
            y = gen.measure(n, m, d, col, supp, vals, w)
            return gen.Instance(n, m, d, k, sseed, col, supp, vals, y, alpha,
                                gen.VALUES_PM1 if kind == "pm1" else gen.VALUES_NORMAL, w)

        for di in active:  # matrices first (cached), then the signals in parallel
            for q in range(problems):
                matrix(di, q)
        with ThreadPoolExecutor(8) as pool:
            insts = list(pool.map(lambda a: draw(*a), [(di, q) for di in active for q in range(problems)]))
        keep = [check_every > 0 and (start + len_done + q) % check_every == 0 for q in range(len(insts))]
        outs = decode(insts, alpha, rule, keep)
        len_done += len(insts)
        nxt = []
        for a, di in enumerate(active):
            ok = 0
            for q in range(problems):
                inst = insts[a * problems + q]
                oc, it, err, x = outs[a * problems + q]
                ok += int(oc == 0 and err <= 1e-6)
                if x is not None:
                    records.append((curve, di, rho, inst, oc, it, x))
            points[di].append((rho, ok))
            if ok > 0 and rho < 1.0 - 1e-9:
                nxt.append(di)
        log(f"[phase] {curve}: rho={rho:.2f} active deltas {len(active)} -> {len(nxt)}")
        active = nxt
        step += 1
    return deltas, points, records, len_done


def phase(args):
    """Phase transitions (Section 5.1 protocol; bands of Section 5.6; degrees
    of Section 5.7) decoded by the batched decoder, one l0_decode_batched
    call per curve and rho step, with sampled instances checked bitwise
    against the oracle."""
    import numpy as np
    import torch

    import paper_1508_01256_amd as l0

    names = list(PHASE_CURVES) if args.phase_curves == "all" else args.phase_curves.split(",")
    for c in names:
        if c not in PHASE_CURVES:
            raise SystemExit(f"unknown curve {c}; known: {', '.join(PHASE_CURVES)}")
    rules = {"L0DEC": l0.L0_RULE_L0DEC, "MODE": l0.L0_RULE_MODE, "SHIFTED_L0DEC": l0.L0_RULE_SHIFTED_L0DEC}
    dev = "cuda"
    gpu_ms = [0.0]
    solves = [0]

    cache = {}  # host array id -> device copy (matrices and weights stay resident per curve)

    def resident(a):
        t = cache.get(id(a))
        if t is None or t[0] is not a:
            t = (a, torch.from_numpy(a).to(dev))
            cache[id(a)] = t
        return t[1]

    def decode(insts, alpha, rule, keep):
        probs = [dict(col_idx=resident(i.col_idx), n=i.n, m=i.m, d=i.d,
                      y=torch.from_numpy(i.y).to(dev), alpha=alpha, max_iter=100, tol=1e-10,
                      x_out=torch.empty(i.n, dtype=torch.float64, device=dev),
                      weights=None if i.w is None else resident(i.w)) for i in insts]
        table = l0.problem_table(probs)
        # the largest LDS word capacity whose schedule fits this degree
        for bt, wc in ((512, 32768), (512, 16384), (256, 8192)):
            opts = l0.l0_batch_opts(rules[rule], 0, bt, wc)
            nb = l0.l0_batch_workspace_bytes(table, opts)
            if nb:
                break
        results = l0.new_results(len(probs), dev)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st = l0.l0_decode_batched(table, opts, results, ws)
        e1.record(stream)
        if st != l0.L0_OK:
            raise RuntimeError(f"l0_decode_batched status {st}")
        torch.cuda.synchronize()
        gpu_ms[0] += e0.elapsed_time(e1)
        solves[0] += len(probs)
        rl = l0.results_list(results)
        out = []
        for i, r, p, kp in zip(insts, rl, probs, keep):
            xt = torch.zeros(i.n, dtype=torch.float64, device=dev)
            if i.k:
                xt[torch.from_numpy(i.supp).to(dev)] = torch.from_numpy(i.vals).to(dev)
            err = float((p["x_out"] - xt).abs().max()) / (float(np.max(np.abs(i.vals))) if i.k else 1.0)
            out.append((r["outcome"], r["iters"], err, p["x_out"].cpu().numpy() if kp else None))
        return out

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    import oracle
    t0 = time.time()
    curves = {}
    checked = agree = 0
    cdt = 0.0
    seen = 0
    for c in names:
        cache.clear()
        deltas, points, records, count = phase_protocol(c, args.phase_n, args.phase_problems, decode, log,
                                                        args.phase_check_every, seen)
        seen += count
        d, alpha, rule, kind, scaled, band = PHASE_CURVES[c]
        star = {}
        for di, pts in points.items():
            rs = [r for r, _ in pts]
            ks = [k for _, k in pts]
            star[round(deltas[di], 4)] = logistic_50(rs, ks, [args.phase_problems] * len(rs))
        curves[c] = star
        orule = {"L0DEC": oracle.RULE_L0DEC, "MODE": oracle.RULE_MODE,
                 "SHIFTED_L0DEC": oracle.RULE_SHIFTED_L0DEC}[rule]
        for (_, di, rho, inst, oc, it, x) in records:
            c0 = time.perf_counter()
            o = oracle.parallel_l0(inst.n, inst.m, inst.d, inst.col_idx, inst.y, alpha, max_iter=100,
                                   tol=1e-10, rule=orule, w=inst.w)
            cdt += time.perf_counter() - c0
            checked += 1
            agree += int(o["outcome"] == oc and o["iters"] == it and np.array_equal(o["x"], x))
        log(f"[phase] {c}: rho*(delta) = " + ", ".join(
            f"{dl:.3f}:{'-' if v is None else f'{v:.3f}'}" for dl, v in star.items()))
    wall = time.time() - t0
    log(f"[phase] {solves[0]} solves, GPU {gpu_ms[0] / 1e3:.2f} s, wall {wall:.1f} s; "
        f"oracle agreement {agree}/{checked}")
    cpu = None
    if not args.no_cpu and checked:
        cpu = {"value": round(checked / cdt, 3), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{checked} instances (every {args.phase_check_every}th decoded), {cdt:.1f} s "
                         f"single thread; {agree}/{checked} bitwise equal to the batched GPU results"}
    out = {
        "metric": "phase transitions: 50% recovery rho*(delta) by logistic fit, batched decoder",
        "value": round(solves[0] / (gpu_ms[0] * 1e-3), 1), "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(gpu_ms[0], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"n={args.phase_n}, delta grid of 24 values, rho from 0.01 in steps of "
                               f"0.01 while any of {args.phase_problems} problems is recovered; "
                               "success = CONVERGED and ||x_hat - x||_inf <= 1e-6 ||x||_inf; "
                               "tol=1e-10, max_iter=100",
                   "curves": {c: dict(zip(("d", "alpha", "rule", "values", "scaled", "band"),
                                          PHASE_CURVES[c])) for c in names}},
        "roofline": None,
        "cpu_baseline": cpu,
        "detail": {"solves": solves[0], "gpu_s": round(gpu_ms[0] / 1e3, 3), "wall_s": round(wall, 1),
                   "oracle_checked": checked, "oracle_agree": agree, "rho_star": curves},
    }
    print(json.dumps(out), flush=True)
    if args.phase_out:
        deltas = phase_deltas()
        with open(args.phase_out, "w") as f:
            f.write("| delta | " + " | ".join(names) + " |\n|---|" + "---|" * len(names) + "\n")
            for dl in deltas:
                key = round(dl, 4)
                cells = [("-" if curves[c][key] is None else f"{curves[c][key]:.3f}") for c in names]
                f.write(f"| {dl:.3f} | " + " | ".join(cells) + " |\n")


if __name__ == "__main__":
    main()
    # every tensor of the run is gone with main's frame: hand the cached
    # device memory back while the runtime is fully up
    release_device()
