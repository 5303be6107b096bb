// Device code of the Parallel-l0 decoder for gfx950.
//
// One solve is a single persistent, cooperatively launched kernel.  Each
// iteration of Algorithm 2 runs as three grid-wide phases:
//   vote     every column j is scored on the same residual r (eq.
//            (selection_l0)); r is staged in LDS when 8m bytes fit, the
//            column-index store is streamed in coalesced 16-byte loads;
//            selected columns apply x_hat_j += omega at once and record the
//            rows they touch;
//   residual each touched row i gets r_i = y_i - sum of x_hat_j over the
//            support columns of row i in ascending j (from +0.0), read from a
//            per-row list of support columns kept sorted; ||r||_0 is updated
//            from the per-row change, counted with wave ballots;
//   control  every workgroup reads the same counters and takes the same
//            decision (converged / stalled / iteration cap).
// Phases are separated by a grid barrier built on one monotonic counter.
#include <hip/hip_runtime.h>

#include <climits>

#include "l0_internal.h"

namespace l0 {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int ld_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier.  Thread 0 of each workgroup publishes its phase's writes
// (release), arrives on a monotonic counter and waits for all workgroups
// (acquire).  A wait longer than `limit` wall-clock ticks raises the abort
// flag instead of spinning forever; every workgroup then leaves the kernel.
__device__ bool grid_sync(Ctrl* c, unsigned& epoch, uint64_t limit) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        epoch += 1;
        const unsigned target = epoch * gridDim.x;
        __threadfence();
        __hip_atomic_fetch_add(&c->bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&c->bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (ld_relaxed(&c->abort)) { ok = 0; break; }
            if (wall_clock64() - t0 > limit) {
                __hip_atomic_store(&c->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Sum of an int over the workgroup; the result is valid in every thread.
__device__ int block_sum(int v) {
    __shared__ int s_part[kWaves];
    __shared__ int s_total;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kWaves; ++w) t += s_part[w];
        s_total = t;
    }
    __syncthreads();
    return s_total;
}

// Number of lanes of this wave with `pred`, in every lane (wave ballot).
__device__ __forceinline__ int wave_count(bool pred) {
    return __popcll(__ballot(pred));
}

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int comp(const v4i& q, int c) {
    return c == 0 ? q.x : c == 1 ? q.y : c == 2 ? q.z : q.w;
}

__device__ __forceinline__ int64_t soa_index(int64_t j, int t, int d) {
    return ((j / kTile) * d + t) * kTile + (j % kTile);
}

__device__ void write_result(const SolveParams& p, int iters, int outcome, int nnz, int support,
                             long long updates) {
    p.res->iters = iters;
    p.res->outcome = outcome;
    p.res->final_nnz = nnz;
    p.res->support_size = support;
    p.res->updates = updates;
    if (p.iters_out) *p.iters_out = (outcome < 16) ? iters : -outcome;
}

// ---------------------------------------------------------------------------
// the score of one column (eq. (selection_l0)) on its gathered values v[0..D)
// ---------------------------------------------------------------------------

// Exact bound test.  With z zeros (|v| <= tau) a candidate's decrease is
// c - z where c counts entries within tau of it.  A zero entry can only be
// within tau of a candidate whose magnitude is at most t2 (~2 tau); without
// such tiny candidates c <= number of nonzeros, otherwise c <= D.  Returns
// true when no candidate can reach a.
template <int D>
__device__ __forceinline__ bool bound_rejects(const double (&v)[D], double tau, double t2, int a,
                                              int rule) {
    int nzc = 0, tiny = 0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const double av = fabs(v[t]);
        const bool nz = av > tau;
        nzc += nz;
        tiny += nz && !(av > t2);
    }
    const int z = D - nzc;
    const int bound = (tiny ? D : nzc) - (rule == L0_RULE_L0DEC ? z : 0);
    return bound < a;
}

// Sorting network (odd-even transposition) on D values.
template <int D>
__device__ __forceinline__ void sort_values(double (&s)[D]) {
#pragma unroll
    for (int round = 0; round < D; ++round) {
#pragma unroll
        for (int i = round & 1; i + 1 < D; i += 2) {
            const double lo = __builtin_fmin(s[i], s[i + 1]);
            const double hi = __builtin_fmax(s[i], s[i + 1]);
            s[i] = lo;
            s[i + 1] = hi;
        }
    }
}

// Necessary condition for a candidate with c >= Q: its entries within tau lie
// in a window of width <= 2 tau (up to one rounding each), i.e. Q consecutive
// sorted values span at most t2.
template <int D, int Q>
__device__ __forceinline__ bool window_q(const double (&s)[D], double t2) {
    bool ok = false;
#pragma unroll
    for (int i = 0; i + Q - 1 < D; ++i) ok |= (s[i + Q - 1] - s[i] <= t2);
    return ok;
}

template <int D, int Q = 2>
__device__ __forceinline__ bool window_pass(const double (&s)[D], int a, double t2) {
    if constexpr (Q > D) {
        return true;
    } else {
        if (a <= Q) return window_q<D, Q>(s, t2);
        return window_pass<D, Q + 1>(s, a, t2);
    }
}

// The score itself, by its definition: for every nonzero candidate v[t],
// c counts the entries u with |v[u] - v[t]| <= tau; the l0-decrease is c - z
// (the frequency rule scores c).  Best score wins, ties go to the smallest
// value.  Returns true (and omega) when the best score reaches a.
template <int D>
__device__ __forceinline__ bool exact_score(const double (&v)[D], double tau, int rule, int a,
                                            double& omega) {
    int z = 0;
#pragma unroll
    for (int u = 0; u < D; ++u) z += !(fabs(v[u]) > tau);
    int top = INT_MIN;
    double w = 0.0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        if (!(fabs(v[t]) > tau)) continue;
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < D; ++u) cnt += !(fabs(v[u] - v[t]) > tau);
        const int score = (rule == L0_RULE_MODE) ? cnt : cnt - z;
        if (top == INT_MIN || score > top || (score == top && v[t] < w)) {
            top = score;
            w = v[t];
        }
    }
    omega = w;
    return top != INT_MIN && top >= a;
}

template <int D>
__device__ void apply_update(const SolveParams& p, int l, int64_t j, double w, const int (&rows)[D]) {
    p.x[j] = p.x[j] + w;
    atomicAdd(&p.tcount[l], 1);
    const uint32_t bit = 1u << (j & 31);
    const uint32_t old = atomicOr(&p.member[j >> 5], bit);
    const bool fresh = (old & bit) == 0;
    if (fresh) atomicAdd(&p.ctrl->support, 1);
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const int i = rows[t];
        if (fresh) {
            const int q = atomicAdd(&p.slot_cnt[i], 1);
            p.slots[p.row_off[i] + q] = static_cast<int>(j);
        }
        if (atomicExch(&p.aff_flag[i], 1) == 0) {
            const int q = atomicAdd(&p.affc[l], 1);
            p.aff_list[q] = i;
        }
    }
}

// Vote phase: each wave takes tiles of kTile columns; lane L holds columns
// 4L..4L+3 of the tile, loading one 16-byte chunk per neighbour plane.
template <int D, bool RL>
__device__ void vote_phase(const SolveParams& p, int l, double tau, double t2, const double* lds_r) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = static_cast<int64_t>(gridDim.x) * kWaves;
    const v4i* soa4 = reinterpret_cast<const v4i*>(p.soa);
    for (int64_t tile = static_cast<int64_t>(blockIdx.x) * kWaves + (threadIdx.x >> 6);
         tile < p.ntiles; tile += nw) {
        v4i idx[D];
#pragma unroll
        for (int t = 0; t < D; ++t) idx[t] = __builtin_nontemporal_load(&soa4[(tile * D + t) * 64 + lane]);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = tile * kTile + lane * 4 + c;
            int rows[D];
            double v[D];
#pragma unroll
            for (int t = 0; t < D; ++t) {
                rows[t] = comp(idx[t], c);
                v[t] = RL ? lds_r[rows[t]] : p.r[rows[t]];
            }
            if (j >= p.n) continue;
            if (bound_rejects<D>(v, tau, t2, p.a, p.rule)) continue;
            double s[D];
#pragma unroll
            for (int t = 0; t < D; ++t) s[t] = v[t];
            sort_values<D>(s);
            if (!window_pass<D>(s, p.a, t2)) continue;
            double w;
            if (exact_score<D>(v, tau, p.rule, p.a, w)) apply_update<D>(p, l, j, w, rows);
        }
    }
}

// r_i = y_i - (sum over the support columns of row i, ascending, of x_hat_j).
// The row's list holds its support columns; entries appended since the last
// visit are merged into the sorted prefix first.
__device__ double row_residual(const SolveParams& p, int i) {
    int* list = p.slots + p.row_off[i];
    const int cnt = p.slot_cnt[i];
    const int done = p.slot_sorted[i];
    for (int q = done; q < cnt; ++q) {
        const int v = list[q];
        int k = q;
        while (k > 0 && list[k - 1] > v) {
            list[k] = list[k - 1];
            --k;
        }
        list[k] = v;
    }
    if (done != cnt) p.slot_sorted[i] = cnt;
    double s = 0.0;
    for (int q = 0; q < cnt; ++q) s += p.x[list[q]];
    return p.y[i] - s;
}

// ---------------------------------------------------------------------------
// the persistent solve kernel
// ---------------------------------------------------------------------------

template <int D, bool RL>
__global__ void __launch_bounds__(kBlock) solve_kernel(SolveParams p, uint64_t limit) {
    extern __shared__ double lds_r[];
    const int tid = threadIdx.x;
    const int64_t gtid = static_cast<int64_t>(blockIdx.x) * kBlock + tid;
    const int64_t gsize = static_cast<int64_t>(gridDim.x) * kBlock;
    Ctrl* c = p.ctrl;
    unsigned epoch = 0;

    // --- init: x_hat, support bitmap, per-row state, max |y|, finiteness
    {
        for (int64_t j = gtid; j < p.n; j += gsize) p.x[j] = p.x_init ? p.x_init[j] : 0.0;
        const int64_t nwords = (p.n + 31) >> 5;
        for (int64_t w = gtid; w < nwords; w += gsize) p.member[w] = 0u;
        double lmax = 0.0;
        int bad = 0;
        for (int64_t i = gtid; i < p.m; i += gsize) {
            const double yi = p.y[i];
            if (!isfinite(yi)) bad = 1;
            else lmax = fmax(lmax, fabs(yi));
            p.slot_cnt[i] = 0;
            p.slot_sorted[i] = 0;
            p.aff_flag[i] = 0;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, off));
        if ((tid & 63) == 0 && lmax > 0.0)
            atomicMax(reinterpret_cast<unsigned long long*>(&c->maxabs_bits),
                      static_cast<unsigned long long>(__double_as_longlong(lmax)));
        if (wave_count(bad != 0) && (tid & 63) == 0) atomicExch(&c->err, L0_DEV_NONFINITE_Y);
        if (gtid == 0 && *p.bad_index) atomicExch(&c->err, L0_DEV_BAD_INDEX);
    }
    if (!grid_sync(c, epoch, limit)) {
        if (gtid == 0) write_result(p, 0, L0_DEV_ABORTED, 0, 0, 0);
        return;
    }
    const int err = ld_relaxed(&c->err);
    if (err) {
        if (gtid == 0) write_result(p, 0, err, 0, 0, 0);
        return;
    }
    const double ymax = __longlong_as_double(static_cast<long long>(
        __hip_atomic_load(&c->maxabs_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    const double tau = (p.tol_mode == L0_TOL_RELATIVE) ? p.tol * ymax : p.tol;
    const double t2 = (tau + tau) * (1.0 + 0x1p-40);

    // --- resume: enter the nonzeros of x_init into the support lists
    if (p.x_init) {
        for (int64_t j = gtid; j < p.n; j += gsize) {
            if (p.x[j] == 0.0) continue;
            atomicOr(&p.member[j >> 5], 1u << (j & 31));
            atomicAdd(&c->support, 1);
            for (int t = 0; t < D; ++t) {
                const int i = p.soa[soa_index(j, t, D)];
                const int q = atomicAdd(&p.slot_cnt[i], 1);
                p.slots[p.row_off[i] + q] = static_cast<int>(j);
            }
        }
        if (!grid_sync(c, epoch, limit)) {
            if (gtid == 0) write_result(p, 0, L0_DEV_ABORTED, 0, 0, 0);
            return;
        }
    }

    // --- r = y - A x_hat and ||r||_0
    {
        int wnz = 0;
        for (int64_t i = gtid; i < p.m; i += gsize) {
            const double ri = p.x_init ? row_residual(p, static_cast<int>(i)) : p.y[i];
            p.r[i] = ri;
            wnz += wave_count(fabs(ri) > tau);
        }
        const int b = block_sum((tid & 63) == 0 ? wnz : 0);
        if (tid == 0 && b) atomicAdd(&c->nnz, b);
    }
    if (!grid_sync(c, epoch, limit)) {
        if (gtid == 0) write_result(p, 0, L0_DEV_ABORTED, 0, 0, 0);
        return;
    }
    int nnz = ld_relaxed(&c->nnz);
    if (gtid == 0 && p.trace) p.trace[0] = nnz;

    int l = 0;
    int outcome;
    long long updates = 0;
    for (;;) {
        if (nnz == 0) { outcome = L0_CONVERGED; break; }
        if (l == p.max_iter) { outcome = L0_MAX_ITER; break; }

        // vote on the same residual for every column
        if (RL) {
            for (int i = tid; i < p.m; i += kBlock) lds_r[i] = p.r[i];
            __syncthreads();
        }
        vote_phase<D, RL>(p, l, tau, t2, lds_r);
        if (!grid_sync(c, epoch, limit)) {
            if (gtid == 0) write_result(p, l, L0_DEV_ABORTED, nnz, 0, updates);
            return;
        }
        const int tc = ld_relaxed(&p.tcount[l]);
        if (tc == 0) { outcome = L0_STALLED; break; }

        // residual update of the touched rows, ||r||_0 by its change
        {
            const int na = ld_relaxed(&p.affc[l]);
            // Each pass of this grid-stride loop has lane 0 of the wave active
            // whenever any lane is, so lane 0 accumulates the wave's change.
            int wdelta = 0;
            for (int64_t q = gtid; q < na; q += gsize) {
                const int i = p.aff_list[q];
                const double rn = row_residual(p, i);
                const bool was = fabs(p.r[i]) > tau;
                const bool now = fabs(rn) > tau;
                p.r[i] = rn;
                p.aff_flag[i] = 0;
                wdelta += wave_count(now && !was) - wave_count(was && !now);
            }
            const int b = block_sum((tid & 63) == 0 ? wdelta : 0);
            if (tid == 0 && b) atomicAdd(&c->nnz, b);
        }
        if (!grid_sync(c, epoch, limit)) {
            if (gtid == 0) write_result(p, l, L0_DEV_ABORTED, nnz, 0, updates);
            return;
        }
        nnz = ld_relaxed(&c->nnz);
        updates += tc;
        ++l;
        if (gtid == 0) {
            if (p.trace) p.trace[l] = nnz;
            if (p.tsize) p.tsize[l - 1] = tc;
        }
    }
    if (gtid == 0) write_result(p, l, outcome, nnz, ld_relaxed(&c->support), updates);
}

// ---------------------------------------------------------------------------
// matrix preparation
// ---------------------------------------------------------------------------

__global__ void zero_ints(int32_t* p, int64_t count) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0;
}

// Repack col_idx (column-major rows) into the tiled neighbour planes, check
// every row index, and count row degrees (LDS histogram when m fits).
template <int D>
__global__ void __launch_bounds__(1024) repack_kernel(const int32_t* col_idx, MatrixView A, int lds_hist) {
    extern __shared__ int hist[];
    const int64_t gtid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t gsize = static_cast<int64_t>(gridDim.x) * blockDim.x;
    if (lds_hist) {
        for (int i = threadIdx.x; i < A.m; i += blockDim.x) hist[i] = 0;
        __syncthreads();
    }
    const int64_t total = A.ntiles * D * kTile;
    int bad = 0;
    for (int64_t o = gtid; o < total; o += gsize) {
        const int64_t tile = o / (D * kTile);
        const int rem = static_cast<int>(o - tile * (D * kTile));
        const int t = rem / kTile;
        const int64_t j = tile * kTile + (rem - t * kTile);
        int row = 0;
        if (j < A.n) {
            row = col_idx[j * D + t];
            if (row < 0 || row >= A.m) {
                bad = 1;
                row = 0;
            } else if (lds_hist) {
                atomicAdd(&hist[row], 1);
            } else {
                atomicAdd(&A.deg[row], 1);
            }
        }
        A.soa[o] = row;
    }
    if (bad) atomicExch(A.bad_index, 1);
    if (lds_hist) {
        __syncthreads();
        for (int i = threadIdx.x; i < A.m; i += blockDim.x)
            if (hist[i]) atomicAdd(&A.deg[i], hist[i]);
    }
}

// row_off = exclusive prefix sum of deg (one workgroup, chunks of 1024).
__global__ void __launch_bounds__(1024) scan_kernel(MatrixView A) {
    __shared__ int s_wave[16];
    __shared__ int s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int base = 0; base < A.m; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < A.m ? A.deg[i] : 0;
        int incl = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        if (lane == 63) s_wave[wid] = incl;
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wid; ++w) before += s_wave[w];
        const int carry = s_carry;
        if (i < A.m) A.row_off[i] = carry + before + incl - v;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = carry + before + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) A.row_off[A.m] = s_carry;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

namespace {

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

uint64_t barrier_limit_ticks() {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;  // 100 MHz
    return static_cast<uint64_t>(khz) * 1000ull * 20ull;  // 20 seconds
}

template <int D>
hipError_t prepare_d(const int32_t* col_idx, const MatrixView& A, hipStream_t s) {
    const int cus = device_cus();
    hipLaunchKernelGGL(zero_ints, dim3(256), dim3(256), 0, s, A.deg, static_cast<int64_t>(A.m));
    hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, A.bad_index, int64_t(1));
    const size_t hist_bytes = static_cast<size_t>(A.m) * sizeof(int);
    const int lds_hist = hist_bytes <= kLdsRBytes ? 1 : 0;
    const size_t lds = lds_hist ? hist_bytes : 0;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&repack_kernel<D>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const int64_t total = A.ntiles * D * kTile;
    int64_t blocks = (total + 1023) / 1024;
    const int64_t cap = static_cast<int64_t>(cus > 0 ? cus : 256) * (lds_hist ? 1 : 8);
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(repack_kernel<D>, dim3(static_cast<unsigned>(blocks)), dim3(1024), lds, s, col_idx, A,
                       lds_hist);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, A);
    return hipGetLastError();
}

template <int D, bool RL>
hipError_t solve_d(const SolveParams& p, hipStream_t s) {
    const void* fn = reinterpret_cast<const void*>(&solve_kernel<D, RL>);
    const size_t lds = RL ? static_cast<size_t>(p.m) * sizeof(double) : 0;
    hipError_t e;
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorLaunchOutOfResources;
    const int cus = device_cus();
    int64_t grid = static_cast<int64_t>(per_cu) * cus;
    // no more workgroups than there are tiles (one wave per tile at least)
    const int64_t want = (p.ntiles + kWaves - 1) / kWaves;
    if (grid > want) grid = want;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(zero_ints, dim3(1), dim3(256), 0, s, reinterpret_cast<int32_t*>(p.ctrl),
                       static_cast<int64_t>(sizeof(Ctrl) / sizeof(int32_t)));
    hipLaunchKernelGGL(zero_ints, dim3(8), dim3(256), 0, s, p.tcount,
                       static_cast<int64_t>(2 * (p.max_iter + 2)));
    SolveParams q = p;
    uint64_t limit = barrier_limit_ticks();
    void* args[] = {&q, &limit};
    return hipLaunchCooperativeKernel(fn, dim3(static_cast<unsigned>(grid)), dim3(kBlock), args,
                                      static_cast<unsigned>(lds), s);
}

template <int D>
hipError_t solve_dispatch_r(const SolveParams& p, hipStream_t s) {
    if (static_cast<size_t>(p.m) * sizeof(double) <= kLdsRBytes) return solve_d<D, true>(p, s);
    return solve_d<D, false>(p, s);
}

template <int D = kDMin>
hipError_t prepare_dispatch(int d, const int32_t* col_idx, const MatrixView& A, hipStream_t s) {
    if constexpr (D > kDMax) {
        return hipErrorInvalidValue;
    } else {
        if (d == D) return prepare_d<D>(col_idx, A, s);
        return prepare_dispatch<D + 1>(d, col_idx, A, s);
    }
}

template <int D = kDMin>
hipError_t solve_dispatch(const SolveParams& p, hipStream_t s) {
    if constexpr (D > kDMax) {
        return hipErrorInvalidValue;
    } else {
        if (p.d == D) return solve_dispatch_r<D>(p, s);
        return solve_dispatch<D + 1>(p, s);
    }
}

}  // namespace

hipError_t launch_prepare(const int32_t* col_idx, const MatrixView& A, int /*check*/, hipStream_t s) {
    return prepare_dispatch(A.d, col_idx, A, s);
}

hipError_t launch_solve(const SolveParams& p, hipStream_t s) { return solve_dispatch(p, s); }

}  // namespace l0
