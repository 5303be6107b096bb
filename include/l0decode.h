/*
 * l0decode — Parallel-l0 expander decoding on AMD Instinct MI355X (gfx950).
 *
 * Problem (Mendoza-Smith & Tanner, "Expander l0-decoding", Algorithm 2 and
 * its Data/Result lines): given the adjacency matrix A of a left d-regular
 * bipartite expander (Definition 2.2: A is m x n, binary, exactly d ones per
 * column), a measurement y = A x of a k-sparse x, and a threshold
 * alpha in (1, d], find x_hat with y = A x_hat by repeating
 *     T <- {(j, omega) : ||r||_0 - ||r - omega a_j||_0 >= alpha}
 *     x_hat_j <- x_hat_j + omega for (j, omega) in T
 *     r <- y - A x_hat
 * where every column j is scored on the same residual r (eq. (selection_l0),
 * Section 4).
 *
 * Conventions shared by every entry point:
 *  - A is passed as col_idx: int32[n*d], column j's d row indices at
 *    col_idx[j*d .. j*d+d), each in [0, m), d distinct rows per column (A is
 *    binary with exactly d ones per column, Definition 2.2).  An index outside
 *    [0, m) ends the solve with L0_DEV_BAD_INDEX, a row listed twice in one
 *    column with L0_DEV_REPEATED_ROW.  Row order inside a column does not
 *    change the result of L0_RULE_L0DEC or L0_RULE_MODE; the shifted rules
 *    try the rows in col_idx order, so for them it does.
 *  - Zero test and equality use tau = tol * max_i |y_i| (or tau = tol with
 *    L0_TOL_ABSOLUTE): an entry v is nonzero iff |v| > tau, and two values
 *    a, b are equal iff |a - b| <= tau (tol = 0 is exact equality).
 *  - The candidates for omega are the nonzero residual values on N(j); the
 *    decrease is an integer, so it is compared with ceil(alpha); a column
 *    takes one update, the smallest candidate among those with the largest
 *    decrease.
 *  - r <- y - A x_hat recomputes each changed r_i as y_i minus the sum of
 *    x_hat_j over the columns j with i in N(j), summed from +0.0 in ascending
 *    j.  Results are deterministic: the same inputs give bitwise the same
 *    x_hat, iteration count and ||r||_0 trace on every run.
 *  - Iterations (Definition 3.1) count residual updates.  The loop ends when
 *    ||r||_0 = 0 (L0_CONVERGED), when no column qualifies (L0_STALLED; r would
 *    never change again) or after max_iter iterations (L0_MAX_ITER).
 *    Non-convergence is an outcome, not an error.
 *  - Column-scaled A (Section 4.3.3: columns multiplied by i.i.d. draws from
 *    a continuous distribution, so that non-dissociated signals such as +-1
 *    values become identifiable): optional weights w, device double[n] with
 *    every w_j > 0 and finite, make column j hold w_j on its d rows.  A
 *    column's scores and chosen residual value r_t are those above (entry u
 *    of r - omega a_j is r_u - r_t once omega = r_t / w_j); the update is
 *    x_hat_j += r_t / w_j, and the residual sums the rounded products
 *    w_j * x_hat_j in ascending j.  Unit weights give bitwise the unweighted
 *    result.  A weight that is not positive and finite ends the solve with
 *    L0_DEV_BAD_WEIGHT before any update.
 *  - All pointers documented as "device" are device memory (hipMalloc or
 *    torch CUDA tensors) owned by the caller unless stated otherwise.  Every
 *    call is asynchronous and ordered on `stream`; outputs are valid after the
 *    stream synchronises.  Argument errors are detected on the host before
 *    any device work and returned as L0_ERR_ARG; problems found by the device
 *    (bad row index, non-finite y) are reported through the outcome.
 */
#ifndef L0DECODE_H
#define L0DECODE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Returned synchronously by every call. */
typedef enum {
    L0_OK = 0,
    L0_ERR_ARG = 1,      /* invalid argument; nothing was enqueued */
    L0_ERR_OOM = 2,      /* device allocation failed */
    L0_ERR_HIP = 3,      /* a HIP runtime call failed */
    L0_ERR_WORKSPACE = 4 /* caller workspace smaller than required */
} l0_status;

/* Written on the device into l0_result.outcome. */
typedef enum {
    L0_CONVERGED = 0,
    L0_STALLED = 1,
    L0_MAX_ITER = 2,
    L0_DEV_BAD_INDEX = 16,   /* a row index outside [0, m) (when checked) */
    L0_DEV_NONFINITE_Y = 17, /* y holds NaN or Inf */
    L0_DEV_ABORTED = 19,     /* the device loop timed out waiting for itself */
    L0_DEV_BAD_WEIGHT = 20,  /* a column weight is zero, negative or not finite */
    L0_DEV_REPEATED_ROW = 21 /* a column lists one row twice (A must be binary, Definition 2.2) */
} l0_outcome;

typedef enum {
    L0_RULE_L0DEC = 0, /* score = l0-decrease ||r||_0 - ||r - omega a_j||_0 (Algorithm 2) */
    L0_RULE_MODE = 1,  /* score = frequency of omega in r_N(j) (parallel-LDDSR, Table 2) */
    /* Shifted Parallel-l0 (Section 4.3.1, Algorithm 3, Theorem 4.8): at vote
     * pass p every column tries one candidate only, the value of r at its
     * (p mod d)-th neighbour in col_idx order (not tried when zero), scored as
     * L0DEC or MODE.  A pass selecting nothing leaves r unchanged and the next
     * pass tries the next position; d such passes in a row end the run as
     * L0_STALLED.  iters, trace and |T| count residual updates as before. */
    L0_RULE_SHIFTED_L0DEC = 2,
    L0_RULE_SHIFTED_MODE = 3
} l0_rule;

typedef enum {
    L0_TOL_RELATIVE = 0, /* tau = tol * max_i |y_i| */
    L0_TOL_ABSOLUTE = 1  /* tau = tol */
} l0_tol_mode;

/* Per-solve summary, written on the device. */
typedef struct {
    int32_t iters;        /* residual updates performed */
    int32_t outcome;      /* l0_outcome */
    int32_t final_nnz;    /* ||r||_0 when the loop ended */
    int32_t support_size; /* columns of x_hat ever updated */
    int64_t updates;      /* total (j, omega) pairs applied over all iterations */
} l0_result;

/* Optional behaviour of l0_decode_ex / l0_solve; NULL means all defaults. */
typedef struct {
    int32_t rule;          /* l0_rule, default L0_RULE_L0DEC */
    int32_t tol_mode;      /* l0_tol_mode, default L0_TOL_RELATIVE */
    int32_t reserved0;     /* must be 0 */
    int32_t reserved1;     /* must be 0 */
    const double* x_init;  /* device double[n] to resume from, or NULL for x_hat = 0 */
    int32_t* trace;        /* device int32[max_iter+1]: ||r||_0 before iteration 1 and after
                              each iteration (entries past iters are left as they were);
                              or NULL */
    int64_t* tsize;        /* device int64[max_iter]: |T| of each iteration, or NULL */
    int64_t* timeline;     /* device int64[6*max_iter + 16] or NULL: device wall-clock ticks
                              (hipDeviceAttributeWallClockRate) seen by workgroup 0: entry 0
                              at kernel start, entry 3*max_iter+7 once every workgroup has
                              started, entry e after the e-th grid-wide barrier
                              for e <= 3*max_iter+6 (later ones, which only a
                              shifted rule's empty passes reach, are not kept);
                              entries 3*max_iter+8+3*l+{0,1,2} when the vote of iteration l
                              has staged the residual, streamed all columns, and scored the
                              columns that passed the filter */
    const double* weights; /* device double[n] column weights of a column-scaled A
                              (Section 4.3.3), or NULL for unit columns */
} l0_opts;

/* Library version string. */
const char* l0_version(void);

/* Human-readable name of a status or outcome code. */
const char* l0_status_string(int32_t code);

/*
 * One-shot Parallel-l0 decode (Algorithm 2).
 *   col_idx  device int32[n*d]      column-index store of A (read only)
 *   n, m, d  sizes; 1 <= n, 2 <= d <= min(m, 20), n*d < 2^31
 *   y        device double[m]       measurement (read only)
 *   alpha    threshold in (1, d]
 *   max_iter >= 0 iterations at most
 *   tol      >= 0, finite; relative zero/equality threshold (see above)
 *   x_out    device double[n]       receives x_hat (zeroed by the call)
 *   iters_out device int32[1]       iterations on CONVERGED/STALLED/MAX_ITER;
 *                                   minus the outcome code on a device error
 * The library allocates and frees its workspace on `stream`
 * (hipMallocAsync/hipFreeAsync).  Every row index is range-checked on the
 * device before use; an index outside [0, m) ends the solve with
 * L0_DEV_BAD_INDEX, a column with a repeated row with L0_DEV_REPEATED_ROW,
 * both leaving x_out zero.
 */
l0_status l0_decode(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, const double* y,
                    double alpha, int32_t max_iter, double tol, double* x_out,
                    int32_t* iters_out, hipStream_t stream);

/*
 * l0_decode without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments and results as l0_decode.  The workspace is
 * a fixed array of L0_NOALLOC_SCRATCH_BYTES in the library's device memory,
 * one per device, held until the process ends; nothing is allocated or freed
 * and no library routine that allocates is called.  Problems whose workspace
 * (l0_noalloc_workspace_bytes) exceeds that size are refused with
 * L0_ERR_WORKSPACE before anything is enqueued (at d = 7 about 3 million
 * columns fit).  Every call on a device uses that device's one array: calls
 * that overlap on one device (several streams, or host threads) race and
 * must not be issued; calls ordered on one stream are safe (each clears what
 * it needs before use).
 */
#define L0_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
l0_status l0_decode_noalloc(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, const double* y,
                            double alpha, int32_t max_iter, double tol, double* x_out,
                            int32_t* iters_out, hipStream_t stream);

/* Bytes of the fixed array l0_decode_noalloc needs for a problem of this
 * shape (0 for invalid sizes); at most L0_NOALLOC_SCRATCH_BYTES is served. */
size_t l0_noalloc_workspace_bytes(int64_t n, int32_t m, int32_t d, int32_t max_iter);

/*
 * Bytes of device workspace l0_decode_ex needs for one problem of this shape
 * (0 for invalid sizes).
 */
size_t l0_workspace_bytes(int64_t n, int32_t m, int32_t d, int32_t max_iter);

/*
 * One-shot decode with options, a device result and caller workspace.
 *   opts       host pointer or NULL
 *   res_out    device l0_result[1]
 *   workspace  device memory of at least l0_workspace_bytes(n, m, d, max_iter),
 *              256-byte aligned; owned by the caller, reusable after the call
 *              completes on `stream`; never allocated or freed here
 * Other arguments as l0_decode.
 */
l0_status l0_decode_ex(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, const double* y,
                       double alpha, int32_t max_iter, double tol, double* x_out,
                       const l0_opts* opts, l0_result* res_out, void* workspace,
                       size_t ws_bytes, hipStream_t stream);

/*
 * A prepared matrix: the column-index store repacked once for coalesced
 * streaming plus per-row capacities, so that many solves on the same A skip
 * the setup.  The handle owns its device memory (allocated here with
 * hipMalloc on the current device) until l0_matrix_destroy.
 */
typedef struct l0_matrix_s* l0_matrix;

/*
 * Build a prepared matrix from col_idx (as l0_decode); the work is enqueued
 * on `stream` and col_idx may be released once the stream has passed it.
 * Row indices are range-checked and each column's rows checked for
 * repeats; solves on a matrix with a bad index end with L0_DEV_BAD_INDEX,
 * on one with a repeated row with L0_DEV_REPEATED_ROW.  *out receives the
 * handle (host object).
 */
l0_status l0_matrix_create(const int32_t* col_idx, int64_t n, int32_t m, int32_t d,
                           l0_matrix* out, hipStream_t stream);

/* Release a prepared matrix (synchronises the device first); NULL is a no-op. */
l0_status l0_matrix_destroy(l0_matrix A);

/* Bytes of workspace l0_solve needs for a prepared matrix. */
size_t l0_solve_workspace_bytes(l0_matrix A, int32_t max_iter);

/*
 * Decode y against a prepared matrix.  Arguments as l0_decode_ex, with the
 * workspace sized by l0_solve_workspace_bytes.
 *
 * The solve (here and in l0_decode / l0_decode_ex) is one persistent kernel
 * of up to one workgroup per compute unit, launched as an ordinary kernel.
 * Its workgroups admit themselves at start: the ones that start become the
 * members, which split the columns and rows and meet at barriers among
 * themselves; a workgroup that cannot start while others run (a device
 * shared with other streams) is left out once the first member has waited
 * a short window (100 us by default), so the solve never waits for it.  The
 * result does not depend on how many workgroups are members.  Solves must
 * not run on one device at the same time as other solves (several streams
 * with member caps, or beside batches): two solves executing at once on
 * disjoint compute units have given results that differ from the oracle.
 * A solve enqueued behind work that holds every compute unit simply waits
 * for it.  A solve enqueues kernels only (no memset, no allocation with a
 * caller workspace), so it may be captured in a HIP graph and replayed.
 */
l0_status l0_solve(l0_matrix A, const double* y, double alpha, int32_t max_iter, double tol,
                   double* x_out, const l0_opts* opts, l0_result* res_out, void* workspace,
                   size_t ws_bytes, hipStream_t stream);

/*
 * Admission settings of the single-instance solve kernel (tests and tuning;
 * process-wide, read when a solve is enqueued).
 *   max_members  > 0: at most this many workgroups become members (the rest
 *                leave at once); <= 0: no cap (one per compute unit); a cap
 *                leaves compute units idle, which other streams' solves must
 *                not use (see l0_solve)
 *   window_us    > 0: how long the first member waits for the others before
 *                closing admission; <= 0: the default, 100 us
 * Results are the same for every setting; only the speed changes.
 * Returns L0_OK.
 */
l0_status l0_set_solve_admission(int32_t max_members, int32_t window_us);

/*
 * Batched decoding: many independent instances (each its own A, y, sizes,
 * alpha, max_iter, tol) of Algorithm 2, as in the phase-transition sweeps of
 * the paper's experiments (Section 5).  One persistent launch per range of
 * column degrees present ([2,4], [5,9], [10,14], [15,20]); workgroups take
 * work from a device counter (largest n*d first), a small instance going to
 * one workgroup and a large one to a team of up to 256 (never more than are
 * resident) that split its columns and rows.  Workspace covers each instance's own scratch.  Each instance's result is
 * bitwise the one l0_decode_ex gives it alone.  Instances must not share
 * x_out buffers.  A call plans its teams for the whole device: calls that
 * overlap on one device (other streams) are not supported, since their
 * teams could wait for members that cannot be scheduled until a 20 s bound
 * aborts them (L0_DEV_ABORTED); the server (l0_server_*) runs its
 * concurrent batches within a share of the device each.
 */
typedef struct {
    const int32_t* col_idx; /* device int32[n*d], as l0_decode */
    int64_t n;
    int32_t m;
    int32_t d;
    const double* y;        /* device double[m] */
    double alpha;           /* in (1, d] */
    int32_t max_iter;       /* >= 0 */
    int32_t reserved;       /* must be 0 */
    double tol;             /* >= 0, finite */
    double* x_out;          /* device double[n], receives x_hat */
    const double* weights;  /* device double[n] column weights (Section 4.3.3), or NULL */
} l0_problem;

/* Launch schedule of l0_decode_batched; zero fields mean "default". */
typedef struct {
    int32_t rule;          /* l0_rule for every instance */
    int32_t tol_mode;      /* l0_tol_mode for every instance */
    int32_t block_threads; /* 256 or 512 threads per workgroup (0: 256) */
    int32_t words_cap;     /* bucket words kept in LDS: 32-bit when m <= words_cap, folded to
                              16 bits when m <= 2*words_cap (0: 8192; else 64..32768) */
    int64_t* timing;       /* optional device int64[8*count]; record i (in ticks of the
                              device's constant 100 MHz clock): [0] start, [1] end,
                              [2] setup, [3] vote, [4] scoring and updates, [5] residual
                              (totals over iterations), [6] workgroup of the team's
                              leader, [7] team size (workgroups on the instance) */
} l0_batch_opts;

/*
 * Bytes of workspace l0_decode_batched needs for `probs[0..count)` (a host
 * array) under `opts` (NULL: enough for every schedule l0_batch_autotune
 * tries).  0 on invalid arguments.  Queries the current device's occupancy.
 */
size_t l0_batch_workspace_bytes(const l0_problem* probs, int32_t count, const l0_batch_opts* opts);

/*
 * Decode probs[0..count) (host array of device pointers; count < 2^23) on
 * `stream`.  results: l0_result[count] (instance i's at i) in device memory
 * or in host memory the device can write (hipHostMalloc): each record's
 * outcome is written last, after a system-scope fence, so a host that stored
 * an impossible outcome there first sees each instance complete, x_out
 * included, as soon as it is.
 * Workspace: device memory of at least l0_batch_workspace_bytes, 256-byte
 * aligned, caller-owned.  Every instance is validated on the host first
 * (L0_ERR_ARG names no instance; check them individually to find it).
 * Row-index (out of range or repeated in a column) and non-finite-y
 * problems are per-instance outcomes.
 */
l0_status l0_decode_batched(const l0_problem* probs, int32_t count, const l0_batch_opts* opts,
                            l0_result* results, void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Pick the schedule for a batch: runs each candidate (workgroup size, LDS
 * word capacity) on a sample of at most 256 of the instances, times it on
 * `stream` (this call synchronises the stream), and writes the fastest into
 * *opts (rule and tol_mode are kept).  The sample's x_out buffers and
 * results[0..256) are overwritten: decode the batch afterwards.
 * Workspace as l0_batch_workspace_bytes(probs, count, NULL).  L0_ERR_WORKSPACE
 * if no candidate fits ws_bytes.
 */
l0_status l0_batch_autotune(const l0_problem* probs, int32_t count, l0_batch_opts* opts,
                            l0_result* results, void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Serving: a decoding server that accepts requests one at a time and decodes
 * them in batches (l0_decode_batched) under a fixed device-memory budget, as
 * a service answering many independent decoding requests would.  Requests
 * waiting when a batch slot is free go into the next batch (first come,
 * first served, as many as fit the free budget); up to max_inflight batches
 * run at once, each on a stream of the server's own.  A request's buffers
 * (col_idx, y, x_out) are the caller's and must stay valid until its
 * completion is returned.  Calls on one server are serialised by a lock;
 * the server uses the device that is current when it is created.
 */
typedef struct l0_server_s* l0_server;

typedef struct {
    size_t budget_bytes;   /* device memory for batch workspaces (allocated at creation) */
    int32_t max_batch;     /* most requests in one batch (0: 1024) */
    int32_t max_inflight;  /* batches running at once, 1..4 (0: 2) */
    l0_batch_opts batch;   /* rule, tol_mode and schedule of every batch (timing must be NULL) */
} l0_server_opts;

typedef struct {
    int64_t id;            /* the caller's request id */
    int32_t status;        /* L0_OK, or the l0_status that failed the request's batch */
    int32_t reserved;
    l0_result result;      /* outcome of the decode (valid when status is L0_OK) */
    double submit_s;       /* server clock (seconds since creation): submission */
    double launch_s;       /* its batch was launched */
    double done_s;         /* the server saw the batch finish (poll or drain) */
} l0_completion;

/* Create a server; L0_ERR_ARG on invalid options, L0_ERR_OOM if the budget
 * cannot be allocated. */
l0_status l0_server_create(const l0_server_opts* opts, l0_server* out);

/* Queue one request (the record is copied).  L0_ERR_ARG on an invalid
 * problem or buffer, L0_ERR_WORKSPACE when it alone needs more than the
 * budget.  Does not launch anything: l0_server_poll does. */
l0_status l0_server_submit(l0_server s, const l0_problem* prob, int64_t id);

/* Make progress without blocking: collect finished batches, launch new ones
 * from the waiting requests, and copy up to cap completions (oldest first)
 * to out.  Returns the number copied, or minus an l0_status on failure. */
int32_t l0_server_poll(l0_server s, l0_completion* out, int32_t cap);

/* Block until every submitted request has completed (launching batches as
 * slots free up); completions stay queued for l0_server_poll. */
l0_status l0_server_drain(l0_server s);

/* Requests submitted whose completion has not yet been returned by poll. */
int64_t l0_server_outstanding(l0_server s);

/* Wait for running batches, free the server.  NULL is accepted. */
l0_status l0_server_destroy(l0_server s);

#ifdef __cplusplus
}
#endif

#endif /* L0DECODE_H */
