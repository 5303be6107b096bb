// Batched Parallel-l0: many independent instances of uneven (n, m, d), as in
// the phase-transition sweeps of the paper's Section 5.
//
// One persistent launch per range of column degrees.  The host cuts each
// instance into T work items (T grows with n*d; T = 1 for most), and the
// workgroups claim items from a device counter in the host-given order
// (largest first), so the T items of an instance go to T workgroups at about
// the same time: the instance's team.  A team runs every phase of Algorithm 2
// on its instance, its members splitting the columns of the vote and the
// rows of the residual update, and synchronises through a counter in the
// instance's control block (a bounded wait).  Every instance has scratch of
// its own size.
//
// The setup pass over the caller's column-index store (degree counts and
// input checks; each wave transposes 64-column groups through LDS, so that a
// lane holds one column's rows) also writes the instance's repacked index
// store: one coalesced plane per neighbour, 16-bit rows when m <= 65536.
// The votes stream that store, several chunks in flight per wave, with no
// transpose.  Row bucket words (l0_filter.h) sit in every member's LDS when
// m fits the launch's word capacity.  Scoring, updates and residual
// recomputation are the single-instance decoder's (l0_filter.h,
// l0_common.h), so every instance's result is bitwise the one it gets alone.
//
// Every device pointer is typed with its address space: a generic pointer
// would compile to flat accesses, whose completion the LDS waits of the vote
// also wait for.
#include <hip/hip_runtime.h>

#include <climits>

#include "l0_batch.h"
#include "l0_common.h"
#include "l0_filter.h"

namespace l0 {

namespace {

template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> global(T* p) {
    return (gptr<T>)p;
}

template <class T>
using lptr = __attribute__((address_space(3))) T*;

// LDS queue of columns passing the filter: kBatchQueue entries split evenly
// over the waves, each wave's segment followed by 64 per-lane discard slots
// (after the vote, the discard slots hold this member's long-list rows).
constexpr int kBatchQueue = 2048;

// Per-instance state (fields named as the single-instance solver's, for
// apply_update / row_residual).
struct BlockState {
    gptr<double> x;
    gptr<const double> y;
    gptr<const double> w;     // column weights, or null for unit columns
    gptr<double> r;
    gptr<uint32_t> rword;
    gptr<uint32_t> member;
    gptr<int32_t> slot_cnt;
    gptr<int32_t> slot_sorted;
    gptr<int32_t> aff_flag;
    gptr<int32_t> aff_list;   // this iteration's touched-row list
    gptr<int32_t> aff_base;   // both lists
    gptr<int32_t> row_off;
    gptr<int32_t> slots;
    gptr<int32_t> overflow;
    gptr<uint32_t> soa;       // repacked index store (batch_chunks of d planes)
};

__device__ BlockState carve(char* base, const l0_problem& P) {
    const InstLayout lay = inst_layout(P.n, P.m, P.d);
    BlockState s{};
    s.x = global(P.x_out);
    s.y = global(P.y);
    s.w = P.weights ? global(P.weights) : nullptr;
    s.r = global(reinterpret_cast<double*>(base + lay.r));
    s.rword = global(reinterpret_cast<uint32_t*>(base + lay.rword));
    s.member = global(reinterpret_cast<uint32_t*>(base + lay.member));
    s.slot_cnt = global(reinterpret_cast<int32_t*>(base + lay.slot_cnt));
    s.slot_sorted = global(reinterpret_cast<int32_t*>(base + lay.slot_sorted));
    s.aff_flag = global(reinterpret_cast<int32_t*>(base + lay.aff_flag));
    s.aff_base = global(reinterpret_cast<int32_t*>(base + lay.aff_list));
    s.aff_list = s.aff_base;
    s.row_off = global(reinterpret_cast<int32_t*>(base + lay.row_off));
    s.slots = global(reinterpret_cast<int32_t*>(base + lay.slots));
    s.overflow = global(reinterpret_cast<int32_t*>(base + lay.overflow));
    s.soa = global(reinterpret_cast<uint32_t*>(base + lay.soa));
    return s;
}

struct Lds {
    lptr<uint32_t> words;  // words_cap entries (also the degree histogram)
    lptr<uint16_t> hwords; // the same memory as 2 * words_cap folded 16-bit words
    lptr<int> stage;       // (blockDim/64) * 64 * D entries
    lptr<int> queue;       // kBatchQueue + (blockDim/64) * 64 entries
    lptr<int> red;         // 16 ints / 8 doubles of reduction scratch
    lptr<int> ctr;         // [0] long rows of this member [1] barrier result
    lptr<int> wq;          // per-wave queue counts (16)
};

// This workgroup's place in its instance's team.
struct Team {
    gptr<TeamCtl> ctl;
    int size;     // T
    int rank;     // 0 .. T-1; rank 0 leads
    int epoch;    // team barriers passed (kept equal in every thread)
    uint64_t limit;
};

// Workgroup-wide sum; valid in every thread.  `red` holds one int per wave.
__device__ int wg_sum(int v, lptr<int> red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < nw; ++w) t += red[w];
    return t;
}

__device__ double wg_max(double v, lptr<double> red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    const int nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t = fmax(t, red[w]);
    return t;
}

// Exclusive prefix sum of a[0..len) (LDS) plus carry into out[0..len);
// returns the new carry.  All threads call it; each takes four consecutive
// entries per round.
__device__ int wg_scan_to(lptr<const int> a, int len, gptr<int32_t> out, int carry, lptr<int> red) {
    constexpr int E = 4;
    const int nw = blockDim.x >> 6, lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int base = 0; base < len; base += blockDim.x * E) {
        const int i0 = base + threadIdx.x * E;
        int v[E], tsum = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            v[e] = i0 + e < len ? a[i0 + e] : 0;
            tsum += v[e];
        }
        int incl = tsum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        __syncthreads();
        if (lane == 63) red[wid] = incl;
        __syncthreads();
        int run = carry + incl - tsum;
        for (int w = 0; w < wid; ++w) run += red[w];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (i0 + e < len) out[i0 + e] = run;
            run += v[e];
        }
        for (int w = 0; w < nw; ++w) carry += red[w];
    }
    return carry;
}

template <class T>
__device__ __forceinline__ T load_agent(gptr<T> p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Team barrier: every member's writes before it are visible to every member
// after it.  Thread 0 of each member arrives on the monotonic counter and
// waits (relaxed polling, bounded by tm.limit device-clock ticks, leaving
// early on the abort flag).  Returns false, in every thread, when the wait
// failed; the flag then tells every member to stop.  A team of one is a
// workgroup barrier.
__device__ bool team_sync(Team& tm, const Lds& L) {
    __syncthreads();
    if (tm.size == 1) return true;
    ++tm.epoch;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        fetch_add(&tm.ctl->bar, 1);
        const int target = tm.size * tm.epoch;
        const uint64_t t0 = wall_clock64();
        int ok = 1;
        while (load_agent(&tm.ctl->bar) < target) {
            if (load_agent(&tm.ctl->abort)) {
                ok = 0;
                break;
            }
            if (wall_clock64() - t0 > tm.limit) {
                __hip_atomic_store(&tm.ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        L.ctr[1] = ok;
    }
    __syncthreads();
    return L.ctr[1] != 0;
}

// Indices of 64-column group g (64*D consecutive ints, lane-strided).  The
// address is clamped into the array, so the load is unconditional (no branch
// for the wait counters to merge over); entries past the end belong to
// columns j >= n, which never pass.
template <int D>
__device__ __forceinline__ void load_group(gptr<const int32_t> col_idx, int64_t g, int64_t nd, int lane,
                                           int (&out)[D]) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int64_t e = g * 64 * D + k * 64 + lane;
        out[k] = col_idx[e < nd ? e : nd - 1];
    }
}

// Neighbour planes of chunk c of the repacked store: one coalesced 32-bit
// load per plane.  The chunk number is clamped into the store, so the load is
// unconditional (no branch for the wait counters to merge over); a clamped
// chunk's columns are >= n and never pass.
template <int D>
__device__ __forceinline__ void load_chunk(gptr<const uint32_t> soa, int64_t c, int64_t last, int lane,
                                           uint32_t (&out)[D]) {
    const gptr<const uint32_t> q = soa + (c < last ? c : last) * (64 * D) + lane;
#pragma unroll
    for (int t = 0; t < D; ++t) out[t] = __builtin_nontemporal_load(q + t * 64);
}

// One vote pass over this member's columns: chunks first, first + stride,
// ... for wave 0, each wave of the member starting one chunk later, kDepth
// chunks in flight per wave.  SPILL = false: each wave appends the columns
// passing the bucket filter to its LDS queue segment and counts them in
// wq[wave], also past the segment's capacity (those are not kept).  SPILL =
// true: every passing column goes to the team's shared global list, counted
// in *spill; this pass runs only after a segment overflowed.
//
// The ordinary pass has no branch and no global write in its loop body:
// either would make the compiler drain all outstanding loads at the loop
// head, serialising the prefetch.  Lanes with nothing to queue store to
// their discard slot instead.  WM: bucket words in LDS as 32-bit words (1)
// or folded 16-bit words (2, twice as many rows), else (0) in global memory.
// R16: 16-bit rows, two columns per lane and chunk.  Columns >= n (the last
// chunk's padding, clamped chunks) gather row 0 and queue nothing.
template <int D, int WM, bool R16, bool SPILL>
__device__ void vote_pass(int64_t n, const BlockState& s, const Lds& L, int a, int rule, int64_t first,
                          int64_t stride, gptr<int> spill) {
    // chunks in flight per wave: about 32 registers of indices
    constexpr int kDepth = D <= 8 ? 4 : (D <= 10 ? 3 : (D <= 16 ? 2 : 1));
    constexpr int kCols = R16 ? 128 : 64;
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    // the wave index is uniform across the wave: a scalar loop (no exec mask)
    const int wid = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int qcap = kBatchQueue / nw;
    const lptr<int> seg = L.queue + wid * (qcap + 64);
    const int64_t nchunks = (n + kCols - 1) / kCols, last = nchunks - 1;
    const gptr<const uint32_t> soa = s.soa;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t c_first = first + wid, c_step = kDepth * stride;
    int count = 0;  // wave-uniform
    // The slots' loads are issued in slot order and each slot is refilled
    // right after it is consumed, so the oldest loads in flight are always
    // the next slot's: every wait is for one slot only.  Scheduling barriers
    // keep the compiler from reordering the batches (a slot issued out of
    // order would make its wait cover the slots after it as well).
    uint32_t buf[kDepth][D];
#pragma unroll
    for (int sl = 0; sl < kDepth; ++sl) {
        load_chunk<D>(soa, c_first + sl * stride, last, lane, buf[sl]);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int64_t c0 = c_first; c0 < nchunks; c0 += c_step) {
#pragma unroll
        for (int sl = 0; sl < kDepth; ++sl) {
            const int64_t c = c0 + sl * stride;
            uint32_t rw[D];
#pragma unroll
            for (int t = 0; t < D; ++t) rw[t] = buf[sl][t];
            // refill this slot (the copy above waited for its loads)
            __builtin_amdgcn_sched_barrier(0);
            load_chunk<D>(soa, c + c_step, last, lane, buf[sl]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int h = 0; h < (R16 ? 2 : 1); ++h) {
                const int64_t j = R16 ? c * kCols + 2 * lane + h : c * kCols + lane;
                const bool in = j < n;
                uint32_t w[D];
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    const uint32_t r = R16 ? (h ? rw[t] >> 16 : rw[t] & 0xFFFFu) : rw[t];
                    const uint32_t row = in ? r : 0u;
                    w[t] = WM == 1 ? L.words[row] : (WM == 2 ? unfold_word(L.hwords[row]) : s.rword[row]);
                }
                const bool pass = bucket_filter<D>(w, a, rule) && in;
                const unsigned long long mask = __ballot(pass);
                if (SPILL) {
                    if (mask) {
                        int qb = 0;
                        if (lane == 0) qb = fetch_add(spill, __popcll(mask));
                        qb = __shfl(qb, 0);
                        if (pass) s.overflow[qb + __popcll(mask & below)] = static_cast<int>(j);
                    }
                } else {
                    const int pos = count + __popcll(mask & below);
                    seg[(pass && pos < qcap) ? pos : qcap + lane] = static_cast<int>(j);
                    count += __popcll(mask);
                }
            }
        }
    }
    if (!SPILL && lane == 0) L.wq[wid] = count;
}

// Exact score of column j (shifted rules: the candidate at position pos).
template <int D>
__device__ void score_column(gptr<const int32_t> col_idx, const BlockState& s, int rule, gptr<TeamCtl> ctl,
                             gptr<IterCounters> ring, int64_t j, double tau, int a, int pos) {
    int rows[D];
    double v[D];
#pragma unroll
    for (int t = 0; t < D; ++t) rows[t] = col_idx[j * D + t];
#pragma unroll
    for (int t = 0; t < D; ++t) v[t] = s.r[rows[t]];
    double om;
    const bool sel = rule_is_shifted(rule) ? exact_score_shifted<D>(v, pos, tau, rule, a, om)
                                           : exact_score<D>(v, tau, rule, a, om);
    if (sel) apply_update<D>(s, &ring->tcount, &ctl->support, &ring->affc, j, column_update(s, j, om), rows);
}

// The vote of one iteration for this member, with the exact scoring of the
// columns it queued in LDS.  Returns true when its queue overflowed: its
// columns then went to the team's shared list, scored after a team barrier.
template <int D, int WM, bool R16>
__device__ bool vote_and_score(gptr<const int32_t> col_idx, int64_t n, const BlockState& s, const Lds& L, int a,
                               int rule, const Team& tm, gptr<IterCounters> ring, double tau, int pos) {
    const int nw = blockDim.x >> 6, qcap = kBatchQueue / nw;
    const int64_t first = static_cast<int64_t>(tm.rank) * nw, stride = static_cast<int64_t>(tm.size) * nw;
    vote_pass<D, WM, R16, false>(n, s, L, a, rule, first, stride, nullptr);
    __syncthreads();
    int total = 0;
    bool over = false;
    for (int w = 0; w < nw; ++w) {
        total += L.wq[w];
        over |= L.wq[w] > qcap;
    }
    if (over) {
        vote_pass<D, WM, R16, true>(n, s, L, a, rule, first, stride, &ring->spill);
        return true;
    }
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        int w = 0, k = q;
        while (k >= L.wq[w]) k -= L.wq[w++];
        score_column<D>(col_idx, s, rule, tm.ctl, ring, L.queue[w * (qcap + 64) + k], tau, a, pos);
    }
    return false;
}

// Store the new residual of row i (and its bucket word); returns the change
// of the row's nonzero indicator.
__device__ __forceinline__ int finish_row(const BlockState& s, const Lds& L, int wm, int i, double rn, double tau,
                                          double inv_w) {
    const bool was = fabs(s.r[i]) > tau;
    const bool now = fabs(rn) > tau;
    s.r[i] = rn;
    const uint32_t w = row_word(rn, tau, inv_w);
    s.rword[i] = w;
    if (wm == 1) L.words[i] = w;
    else if (wm == 2) L.hwords[i] = fold_word(w);
    s.aff_flag[i] = 0;
    return static_cast<int>(now) - static_cast<int>(was);
}

// Longest support list sorted in LDS; longer ones are sorted in place in
// global memory.
constexpr int kLongList = 1024;
static_assert(kLongList + 2 * 512 <= kBatchQueue, "long-list buffers live in the queue region");

// Ascending sort of buf[0..cnt) by the whole workgroup: the bitonic network
// in its direction-free form (each block of k first compares mirrored pairs
// t and t ^ (k - 1), then the half-cleaners t and t ^ j), with pairs past
// cnt skipped, which acts as padding with +infinity.  GLOBAL: buf is in
// global memory; every step then ends with an acquire of the other threads'
// stores.
template <bool GLOBAL, class Ptr>
__device__ void wg_sort(Ptr buf, int cnt) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    int p2 = 1;
    while (p2 < cnt) p2 <<= 1;
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int mask = (j == (k >> 1)) ? k - 1 : j;
            for (int t = tid; t < p2; t += nthr) {
                const int l = t ^ mask;
                if (l > t && l < cnt) {
                    const int a = buf[t], b = buf[l];
                    if (a > b) {
                        buf[t] = b;
                        buf[l] = a;
                    }
                }
            }
            __syncthreads();
            if (GLOBAL) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
}

// At most this many entries appended since a long list was last sorted are
// merged into its sorted prefix by rank; more are sorted from scratch.
constexpr int kMergeNew = 256;

// row_residual for one row with a long support list, computed by the whole
// workgroup (every thread calls it; the result is valid in thread 0): the
// list is sorted (in LDS when it fits, else in place) when it has unsorted
// entries, then the column terms are gathered 512 entries at a time into LDS
// and thread 0 adds them in ascending j from +0.0.  A list in LDS whose
// sorted prefix has a few new entries after it is merged instead: the
// column ids are distinct, so entry v goes to position (prefix entries
// below v) + (new entries below v), one thread per entry.
__device__ double long_row_residual(const BlockState& s, const Lds& L, int i) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int cnt = s.slot_cnt[i];
    const auto list = s.slots + s.row_off[i];
    const int done = s.slot_sorted[i];
    const bool sorted = done == cnt;
    const bool in_lds = cnt <= kLongList;
    const lptr<int> sb = L.queue;
    const lptr<double> xb = (lptr<double>)(L.queue + kLongList);
    if (in_lds) {
        for (int t = tid; t < cnt; t += nthr) sb[t] = list[t];
        __syncthreads();
        if (!sorted && done > 0 && cnt - done <= kMergeNew) {
            const lptr<int> db = (lptr<int>)xb;  // kLongList ints, free until the gather
            for (int t = tid; t < cnt; t += nthr) {
                const int v = sb[t];
                int below = 0;
                for (int u = done; u < cnt; ++u) below += sb[u] < v;
                if (t < done) {
                    below += t;
                } else {
                    int lo = 0, hi = done;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (sb[mid] < v) lo = mid + 1;
                        else hi = mid;
                    }
                    below += lo;
                }
                db[below] = v;
            }
            __syncthreads();
            for (int t = tid; t < cnt; t += nthr) {
                const int v = db[t];
                sb[t] = v;
                list[t] = v;
            }
        } else if (!sorted) {
            wg_sort<false>(sb, cnt);
            for (int t = tid; t < cnt; t += nthr) list[t] = sb[t];
        }
    } else if (!sorted) {
        wg_sort<true>(list, cnt);
    }
    __syncthreads();
    if (tid == 0 && !sorted) s.slot_sorted[i] = cnt;
    double sum = 0.0;
    for (int c0 = 0; c0 < cnt; c0 += 512) {
        const int len = min(512, cnt - c0);
        for (int t = tid; t < len; t += nthr) xb[t] = column_term(s, in_lds ? sb[c0 + t] : list[c0 + t]);
        __syncthreads();
        if (tid == 0)
            for (int t = 0; t < len; ++t) sum += xb[t];
        __syncthreads();
    }
    return s.y[i] - sum;
}

// Support lists of at most this many entries are summed by one wave.
constexpr int kWaveList = 256;

// Ascending bitonic sort of kWaveList ints held by one wave, entry e in
// v[e / 64] of lane e % 64; pairs one register apart are exchanged within
// the lane, pairs within a register across lanes.
__device__ __forceinline__ void wave_sort(int (&v)[kWaveList / 64]) {
    constexpr int K = kWaveList / 64;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int size = 2; size <= kWaveList; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= 64) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int kp = k ^ (stride >> 6);
                    if (kp > k) {
                        const bool up = ((k * 64 + lane) & size) == 0;
                        const int a = v[k], b = v[kp];
                        v[k] = up ? min(a, b) : max(a, b);
                        v[kp] = up ? max(a, b) : min(a, b);
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int other = __shfl_xor(v[k], stride);
                    const bool up = ((k * 64 + lane) & size) == 0;
                    const bool lower = (lane & stride) == 0;
                    v[k] = (lower == up) ? min(v[k], other) : max(v[k], other);
                }
            }
        }
    }
}

__device__ __forceinline__ double read_lane(double v, int l) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xFFFFFFFFu), l));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), l));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// row_residual for one row whose support list has at most kWaveList
// entries, computed by one wave (every lane calls it; the result is valid in
// every lane): the list is sorted in registers (and written back) when it
// has unsorted entries, each lane gathers the column terms of its entries,
// and the terms are added in ascending j from +0.0, lane by lane.
__device__ __noinline__ double wave_row_residual(const BlockState& s, int i) {
    constexpr int K = kWaveList / 64;
    const int lane = threadIdx.x & 63;
    const int cnt = s.slot_cnt[i];
    const auto list = s.slots + s.row_off[i];
    int v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = k * 64 + lane < cnt ? list[k * 64 + lane] : INT_MAX;
    if (s.slot_sorted[i] != cnt) {
        wave_sort(v);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k * 64 + lane < cnt) list[k * 64 + lane] = v[k];
        if (lane == 0) s.slot_sorted[i] = cnt;
    }
    double xv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) xv[k] = k * 64 + lane < cnt ? column_term(s, v[k]) : 0.0;
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int len = min(64, cnt - k * 64);
        for (int l = 0; l < len; ++l) sum += read_lane(xv[k], l);
    }
    return s.y[i] - sum;
}

// The outcome is written last, after a system-scope fence: a host polling
// results in host-mapped memory sees a complete record (and a finished
// x_hat) once the outcome is no longer the value it stored there.
__device__ void write_result(gptr<l0_result> res, int iters, int outcome, int nnz, int support,
                             long long updates) {
    res->iters = iters;
    res->final_nnz = nnz;
    res->support_size = support;
    res->updates = updates;
    __threadfence_system();
    __hip_atomic_store(&res->outcome, outcome, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Device clock (constant 100 MHz), read by thread 0 for the optional
// per-instance timing record.
__device__ __forceinline__ int64_t stamp() {
    return static_cast<int64_t>(wall_clock64());
}

// Groups of 64 columns in flight per wave in the setup passes.
template <int D>
struct SetupDepth {
    static constexpr int kH = D <= 8 ? 4 : (D <= 12 ? 3 : 2);
};

// Rows r[0..D) of lane `lane`'s column in group g into the repacked store,
// with raw buffer stores over the group's own part: a group past the last
// (ngroups) has an empty range, so every call issues D stores whatever g is
// and the waits for the index loads count them exactly.
// A value the whole wave holds, in scalar registers (a buffer resource built
// from it then needs no per-lane loop).
__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

template <int D>
__device__ __forceinline__ void store_group_rows(gptr<uint32_t> soa, int64_t g, int64_t ngroups, bool r16, int lane,
                                                 const int (&r)[D]) {
    constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit dwords (gfx9)
    const int bytes = __builtin_amdgcn_readfirstlane(g < ngroups ? D * 256 : 0);
    if (r16) {
        char* base = (char*)wave_uniform(reinterpret_cast<uint64_t>((char*)soa + (g >> 1) * (256 * D) + (g & 1) * 128));
        const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, kRsrcWord3);
#pragma unroll
        for (int t = 0; t < D; ++t)
            __builtin_amdgcn_raw_buffer_store_b16(static_cast<unsigned short>(r[t]), rsrc, (t * 128 + lane) * 2, 0, 0);
    } else {
        char* base = (char*)wave_uniform(reinterpret_cast<uint64_t>((char*)soa + g * (256 * D)));
        const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, kRsrcWord3);
#pragma unroll
        for (int t = 0; t < D; ++t) __builtin_amdgcn_raw_buffer_store_b32(r[t], rsrc, (t * 64 + lane) * 4, 0, 0);
    }
}

// First setup pass over this wave's 64-column groups (g_first, g_first +
// g_stride, ...) of the caller's column-index store: each group's D
// coalesced loads are transposed through the wave's LDS staging area, so that
// a lane holds one column's rows; every row is range-checked, no column may
// list a row twice (bits into *bad), the rows go to the repacked store, and
// rows below len are counted in hist.  kH groups in flight, in slots taking
// turns; slots past the last group load a clamped address and do nothing.
template <int D>
__device__ void setup_first_pass(gptr<const int32_t> col_idx, int64_t n, int m, const BlockState& s,
                                 lptr<int> stage, lptr<int> hist, int len, int64_t g_first, int64_t g_stride,
                                 bool r16, int& bad) {
    constexpr int kH = SetupDepth<D>::kH;
    const int lane = threadIdx.x & 63;
    const int64_t nd = n * D, ngroups = (n + 63) >> 6;
    // (slot order kept as in vote_pass)
    int buf[kH][D];
#pragma unroll
    for (int sl = 0; sl < kH; ++sl) {
        load_group<D>(col_idx, g_first + sl * g_stride, nd, lane, buf[sl]);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int64_t g0 = g_first; g0 < ngroups; g0 += kH * g_stride) {
#pragma unroll
        for (int sl = 0; sl < kH; ++sl) {
            const int64_t g = g0 + sl * g_stride;
#pragma unroll
            for (int k = 0; k < D; ++k) stage[k * 64 + lane] = buf[sl][k];
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
            __builtin_amdgcn_wave_barrier();
            int r[D];
#pragma unroll
            for (int t = 0; t < D; ++t) r[t] = stage[lane * D + t];
            // every lane has read its column before the next group's stores
            __builtin_amdgcn_s_waitcnt(0xC07F);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_sched_barrier(0);
            load_group<D>(col_idx, g + kH * g_stride, nd, lane, buf[sl]);
            __builtin_amdgcn_sched_barrier(0);
            const bool col = g * 64 + lane < n;  // slots past the last column hold no column
            if (col) {
#pragma unroll
                for (int t = 0; t < D; ++t)
                    if (r[t] < 0 || r[t] >= m) bad |= kErrBadIndex;
                if (has_repeat<D>(r)) bad |= kErrRepeatedRow;
            }
            // (rows of lanes past the last column are padding; a bad index
            // is stored truncated, and the instance ends with an input error
            // before any vote)
            store_group_rows<D>(s.soa, g, ngroups, r16, lane, r);
#pragma unroll
            for (int t = 0; t < D; ++t)
                if (col && r[t] >= 0 && r[t] < len) fetch_add(&hist[r[t]], 1);
        }
    }
    // the stores are done before this wave reads them back (later passes)
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// A later setup pass (rows lo .. lo+len-1 counted in hist): each wave reads
// back the rows of its own groups from the repacked store (written by this
// wave in the first pass), D coalesced loads per group, kH groups in flight.
template <int D>
__device__ void setup_count_pass(int64_t n, const BlockState& s, lptr<int> hist, int lo, int len, int64_t g_first,
                                 int64_t g_stride, bool r16) {
    constexpr int kH = SetupDepth<D>::kH;
    const int lane = threadIdx.x & 63;
    const int64_t ngroups = (n + 63) >> 6;
    auto load = [&](int64_t g, uint32_t (&out)[D]) {
        const int64_t gc = g < ngroups ? g : ngroups - 1;
        if (r16) {
            const gptr<const uint16_t> q = (gptr<const uint16_t>)s.soa + (gc >> 1) * (128 * D) + (gc & 1) * 64 + lane;
#pragma unroll
            for (int t = 0; t < D; ++t) out[t] = q[t * 128];
        } else {
            const gptr<const uint32_t> q = s.soa + gc * (64 * D) + lane;
#pragma unroll
            for (int t = 0; t < D; ++t) out[t] = q[t * 64];
        }
    };
    uint32_t buf[kH][D];
#pragma unroll
    for (int sl = 0; sl < kH; ++sl) {
        load(g_first + sl * g_stride, buf[sl]);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int64_t g0 = g_first; g0 < ngroups; g0 += kH * g_stride) {
#pragma unroll
        for (int sl = 0; sl < kH; ++sl) {
            const int64_t g = g0 + sl * g_stride;
            uint32_t r[D];
#pragma unroll
            for (int t = 0; t < D; ++t) r[t] = buf[sl][t];
            __builtin_amdgcn_sched_barrier(0);
            load(g + kH * g_stride, buf[sl]);
            __builtin_amdgcn_sched_barrier(0);
            const bool col = g * 64 + lane < n;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                const int rel = static_cast<int>(r[t]) - lo;
                if (col && rel >= 0 && rel < len) fetch_add(&hist[rel], 1);
            }
        }
    }
}

// One member's part of decoding instance P.  Not inlined: each degree gets
// its own register allocation inside the range kernels (the call costs one
// register save per work item).
template <int D>
__device__ __noinline__ void solve_instance(const l0_problem& P_in, const BatchParams& bp_in, const Lds& L_in,
                                            int inst, int rank, int tsize) {
    // copies of the arguments: read once, then never reloaded in the loops
    // (through the references they could alias any store)
    const l0_problem P = P_in;
    const BatchParams bp = bp_in;
    const Lds L = L_in;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool lead = rank == 0;
    Team tm;
    tm.ctl = global(bp.ctl + inst);
    tm.size = tsize;
    tm.rank = rank;
    tm.epoch = 0;
    tm.limit = bp.wait_limit;
    const gptr<l0_result> res = global(bp.results + inst);
    const gptr<int64_t> tim = (bp.timing && lead) ? global(bp.timing + 8 * static_cast<int64_t>(inst)) : nullptr;
    BlockState s = carve(bp.scratch + bp.inst_off[inst], P);
    const gptr<const int32_t> col_idx = global(P.col_idx);
    const int64_t n = P.n;
    const int m = P.m;
    // bucket words in LDS: 32-bit when m fits the word capacity, folded to
    // 16 bits when it fits twice over, else read from global memory
    const int wm = m <= bp.words_cap ? 1 : (m <= 2 * bp.words_cap ? 2 : 0);
    const bool r16 = batch_rows16(m);
    const int64_t gt = static_cast<int64_t>(rank) * nthr + tid, gstep = static_cast<int64_t>(tsize) * nthr;

    // --- init, split over the team: x_hat = 0, support bitmap, per-row
    //     state, r = y; max |y|, non-finite y and unusable column weights
    //     into the control block
    int bad_w = 0;
    for (int64_t j = gt; j < n; j += gstep) {
        s.x[j] = 0.0;
        if (s.w && !weight_ok(s.w[j])) bad_w = 1;
    }
    for (int64_t w = gt; w < ((n + 31) >> 5); w += gstep) s.member[w] = 0u;
    double lmax = 0.0;
    int bad = 0;
    {
        constexpr int U = 4;  // y loads in flight per thread
        for (int64_t i0 = gt; i0 < m; i0 += U * gstep) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = s.y[min(i0 + u * gstep, static_cast<int64_t>(m) - 1)];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + u * gstep;
                if (i < m) {
                    const double yi = v[u];
                    if (!isfinite(yi)) bad = 1;
                    else lmax = fmax(lmax, fabs(yi));
                    s.r[i] = yi;
                    s.slot_cnt[i] = 0;
                    s.slot_sorted[i] = 0;
                    s.aff_flag[i] = 0;
                }
            }
        }
    }
    lmax = wg_max(lmax, (lptr<double>)L.red);
    bad = wg_sum(bad, L.red);
    bad_w = wg_sum(bad_w, L.red);
    if (tid == 0) {
        __hip_atomic_fetch_max(&tm.ctl->ymax_bits, static_cast<unsigned long long>(__double_as_longlong(lmax)),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int flags = (bad ? kErrNonfiniteY : 0) | (bad_w ? kErrBadWeight : 0);
        if (flags) __hip_atomic_fetch_or(&tm.ctl->bad, flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    bool alive = team_sync(tm, L);

    // --- row degrees -> row_off (exclusive scan), counted in LDS one range
    //     of words_cap rows at a time over this member's share of the
    //     columns.  The first pass reads the caller's store (and checks it
    //     and writes the repacked store, see setup_first_pass), later ones
    //     read the repacked store back.  A team adds its counts in slot_cnt;
    //     each member then scans a slice of the rows, and the slices are
    //     joined by their totals.
    const int hcap = bp.words_cap;
    const lptr<int> hist = (lptr<int>)L.words;
    const int lane = tid & 63, nw = nthr >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const lptr<int> stage = L.stage + wid * (64 * D);
    const int64_t g_first = static_cast<int64_t>(rank) * nw + wid, g_stride = static_cast<int64_t>(tsize) * nw;
    int bad_idx = 0;
    int carry = 0;
    for (int lo = 0; alive && lo < m; lo += hcap) {
        const int len = min(hcap, m - lo);
        for (int i = tid; i < len; i += nthr) hist[i] = 0;
        __syncthreads();
        if (lo == 0)
            setup_first_pass<D>(col_idx, n, m, s, stage, hist, len, g_first, g_stride, r16, bad_idx);
        else
            setup_count_pass<D>(n, s, hist, lo, len, g_first, g_stride, r16);
        __syncthreads();
        if (tsize == 1) {
            carry = wg_scan_to(hist, len, s.row_off + lo, carry, L.red);
        } else {
            for (int i = tid; i < len; i += nthr)
                if (hist[i]) fetch_add(&s.slot_cnt[lo + i], hist[i]);
        }
        __syncthreads();
    }
    // the error bits of every wave (an OR of per-wave ORs)
    {
        int wbad = bad_idx;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) wbad |= __shfl_xor(wbad, off);
        if (lane == 0 && wbad) __hip_atomic_fetch_or(&tm.ctl->bad, wbad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tsize > 1) {
        // member `rank` scans rows [r0, r1) from zero and posts the slice
        // total (in the instance's overflow list, unused until the votes);
        // after a team barrier it adds the totals of the slices before it
        alive = alive && team_sync(tm, L);
        const int r0 = static_cast<int>(static_cast<int64_t>(m) * rank / tsize);
        const int r1 = static_cast<int>(static_cast<int64_t>(m) * (rank + 1) / tsize);
        if (alive) {
            const lptr<int> chunk = (lptr<int>)L.words;
            int c2 = 0;
            for (int lo = r0; lo < r1; lo += hcap) {
                const int len = min(hcap, r1 - lo);
                for (int i = tid; i < len; i += nthr) {
                    chunk[i] = load_agent(&s.slot_cnt[lo + i]);
                    s.slot_cnt[lo + i] = 0;
                }
                __syncthreads();
                c2 = wg_scan_to(chunk, len, s.row_off + lo, c2, L.red);
                __syncthreads();
            }
            if (tid == 0) s.overflow[rank] = c2;
        }
        alive = alive && team_sync(tm, L);
        if (alive) {
            // (tsize <= kMaxTeam <= blockDim.x: one slice total per thread)
            const int base = wg_sum(tid < rank ? load_agent(&s.overflow[tid]) : 0, L.red);
            if (base)
                for (int i = r0 + tid; i < r1; i += nthr) s.row_off[i] += base;
            if (rank == tsize - 1 && tid == 0) carry = base + load_agent(&s.overflow[rank]);
        }
    }
    if (rank == tsize - 1 && tid == 0) s.row_off[m] = carry;
    alive = alive && team_sync(tm, L);
    const int flags = load_agent(&tm.ctl->bad);
    if (!alive || flags) {
        if (lead && tid == 0)
            write_result(res, 0, !alive ? L0_DEV_ABORTED : error_outcome(flags), 0, 0, 0);
        __syncthreads();
        return;
    }
    const double ymax = __longlong_as_double(static_cast<long long>(load_agent(&tm.ctl->ymax_bits)));
    const double tau = (bp.tol_mode == L0_TOL_RELATIVE) ? P.tol * ymax : P.tol;
    const double inv_w = 1.0 / bucket_width(tau, ymax);
    const int a = static_cast<int>(ceil(P.alpha));
    // bucket words: every member keeps all of them in LDS (when m fits);
    // the global copy and ||y||_0 are split over the team
    // (y in rounds of U loads in flight per thread)
    constexpr int U = 8;
    if (wm) {
        for (int i0 = tid; i0 < m; i0 += U * nthr) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = s.y[min(i0 + u * nthr, m - 1)];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * nthr;
                if (i < m) {
                    const uint32_t w = row_word(v[u], tau, inv_w);
                    if (wm == 1) L.words[i] = w;
                    else L.hwords[i] = fold_word(w);
                }
            }
        }
    }
    int nzc = 0;
    for (int64_t i0 = gt; i0 < m; i0 += U * gstep) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = s.y[min(i0 + u * gstep, static_cast<int64_t>(m) - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * gstep;
            if (i < m) {
                s.rword[i] = row_word(v[u], tau, inv_w);
                nzc += fabs(v[u]) > tau;
            }
        }
    }
    nzc = wg_sum(nzc, L.red);
    if (tid == 0) fetch_add(&tm.ctl->nnz, nzc);
    alive = team_sync(tm, L);
    int nnz = load_agent(&tm.ctl->nnz);
    int64_t t_last = 0, t_vote = 0, t_score = 0, t_resid = 0;
    if (tim && tid == 0) {
        t_last = stamp();
        tim[2] = t_last - tim[0];
    }

    // Counters and touched-row lists go by vote pass, which differs from the
    // iteration under a shifted rule: a pass selecting nothing is followed by
    // another (the next position), and D such passes in a row stall the run.
    int l = 0, pass = 0, empty = 0, outcome = L0_DEV_ABORTED;
    const bool shifted = rule_is_shifted(bp.rule);
    long long updates = 0;
    while (alive) {
        if (nnz == 0) { outcome = L0_CONVERGED; break; }
        if (l == P.max_iter) { outcome = L0_MAX_ITER; break; }
        const gptr<IterCounters> ring = &tm.ctl->ring[pass % 3];
        const int pos = pass % D;
        s.aff_list = s.aff_base + (pass & 1) * m;
        if (tid == 0) L.ctr[0] = 0;
        __syncthreads();

        // vote and exact scoring of this member's columns (Jacobi updates)
        // (16-bit rows whenever the words are in LDS: m <= 2 * words_cap <= 65536)
        if (wm == 1) vote_and_score<D, 1, true>(col_idx, n, s, L, a, bp.rule, tm, ring, tau, pos);
        else if (wm == 2) vote_and_score<D, 2, true>(col_idx, n, s, L, a, bp.rule, tm, ring, tau, pos);
        else if (r16) vote_and_score<D, 0, true>(col_idx, n, s, L, a, bp.rule, tm, ring, tau, pos);
        else vote_and_score<D, 0, false>(col_idx, n, s, L, a, bp.rule, tm, ring, tau, pos);
        if (lead && tid == 0) {
            const gptr<IterCounters> next = &tm.ctl->ring[(pass + 1) % 3];
            next->tcount = 0;
            next->affc = 0;
            next->spill = 0;
            next->delta = 0;
        }
        if (tim && tid == 0) {
            const int64_t t = stamp();
            t_vote += t - t_last;
            t_last = t;
        }
        if (!(alive = team_sync(tm, L))) break;
        // columns of overflowed queues, scored by the whole team
        const int nsp = load_agent(&ring->spill);
        if (nsp > 0) {
            for (int64_t q = gt; q < nsp; q += gstep)
                score_column<D>(col_idx, s, bp.rule, tm.ctl, ring, s.overflow[q], tau, a, pos);
            if (!(alive = team_sync(tm, L))) break;
        }
        // support-list counts were raised by device-scope atomics: acquire
        // before reading them.  A team of one workgroup needs no cache
        // maintenance (its waves share one CU's caches; the workgroup
        // barrier orders them), and an agent-scope acquire would invalidate
        // the L2 of its XCD for every instance decoding there, every
        // iteration (sweep 14.24 -> 13.92 ms without it)
        if (tsize > 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (tim && tid == 0) {
            const int64_t t = stamp();
            t_score += t - t_last;
            t_last = t;
        }
        ++pass;
        const int tc = load_agent(&ring->tcount);
        if (tc == 0) {
            if (shifted && ++empty < D) continue;
            outcome = L0_STALLED;
            break;
        }
        empty = 0;

        // residual update of the touched rows, split over the team; short
        // support lists one row per thread, longer ones one row per wave
        // afterwards, the longest by this whole workgroup; ||r||_0 by its
        // change
        const int na = load_agent(&ring->affc);
        const int long_cap = (nthr >> 6) * 64;
        const lptr<int> long_rows = L.queue + kBatchQueue;
        int delta = 0;
        // rows dealt round-robin over the team's members (entry q to member
        // q mod tsize), so that a short list is spread over the team
        for (int64_t q = static_cast<int64_t>(tid) * tsize + rank; q < na; q += gstep) {
            const int i = s.aff_list[q];
            const int cnt = s.slot_cnt[i];
            if (cnt <= kShortList) {
                delta += finish_row(s, L, wm, i, row_residual_any(s, i, cnt), tau, inv_w);
            } else {
                const int k = fetch_add(&L.ctr[0], 1);
                if (k < long_cap) long_rows[k] = i;
                else delta += finish_row(s, L, wm, i, row_residual(s, i), tau, inv_w);
            }
        }
        __syncthreads();
        const int nl = min(L.ctr[0], long_cap);
        for (int li = tid >> 6; li < nl; li += nthr >> 6) {
            const int i = long_rows[li];
            if (s.slot_cnt[i] > kWaveList) continue;  // uniform across the wave
            const double rn = wave_row_residual(s, i);
            if ((tid & 63) == 0) {
                delta += finish_row(s, L, wm, i, rn, tau, inv_w);
                long_rows[li] = -1;
            }
        }
        __syncthreads();
        for (int li = 0; li < nl; ++li) {
            const int i = long_rows[li];
            if (i < 0) continue;  // done by a wave (uniform across the workgroup)
            const double rn = long_row_residual(s, L, i);
            if (tid == 0) delta += finish_row(s, L, wm, i, rn, tau, inv_w);
        }
        delta = wg_sum(delta, L.red);
        if (tid == 0) fetch_add(&ring->delta, delta);
        if (!(alive = team_sync(tm, L))) break;
        nnz += load_agent(&ring->delta);
        updates += tc;
        ++l;
        // the other members' rows: refresh their words in this LDS copy
        if (wm && tsize > 1) {
            for (int q = tid; q < na; q += nthr) {
                const int i = s.aff_list[q];
                if (wm == 1) L.words[i] = s.rword[i];
                else L.hwords[i] = fold_word(s.rword[i]);
            }
        }
        __syncthreads();
        if (tim && tid == 0) {
            const int64_t t = stamp();
            t_resid += t - t_last;
            t_last = t;
        }
    }
    if (lead && tid == 0) {
        if (!alive) outcome = L0_DEV_ABORTED;
        write_result(res, l, outcome, nnz, load_agent(&tm.ctl->support), updates);
        if (tim) {
            tim[3] = t_vote;
            tim[4] = t_score;
            tim[5] = t_resid;
        }
    }
    __syncthreads();
}

template <int D, int DHI>
__device__ void solve_dispatch(const l0_problem& P, const BatchParams& bp, const Lds& L, int inst, int rank,
                               int tsize) {
    if constexpr (D > DHI) {
        return;
    } else {
        if (P.d == D) solve_instance<D>(P, bp, L, inst, rank, tsize);
        else solve_dispatch<D + 1, DHI>(P, bp, L, inst, rank, tsize);
    }
}

// One kernel per range of degrees [DLO, DHI] (kBatchRanges): instances of
// all degrees of a range share one persistent launch, so a sweep over
// several degrees is not split into launches that each wait for their
// slowest instance.
template <int BS, int DLO, int DHI>
__global__ void __launch_bounds__(BS) batch_kernel(BatchParams bp) {
    extern __shared__ uint32_t lds[];
    __shared__ double red[16];  // reduction scratch, read as int or double
    __shared__ int ctr[8];
    __shared__ int wq[16];
    __shared__ int s_item;
    Lds L;
    L.words = (lptr<uint32_t>)lds;
    L.hwords = (lptr<uint16_t>)lds;
    L.stage = (lptr<int>)(lds + bp.words_cap);
    L.queue = L.stage + (BS / 64) * 64 * bp.stage_d;
    L.red = (lptr<int>)red;
    L.ctr = (lptr<int>)ctr;
    L.wq = (lptr<int>)wq;
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned q = atomicAdd(bp.next, 1u);
            s_item = q < static_cast<unsigned>(bp.count) ? bp.items[q] : -1;
        }
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item < 0) break;
        const int inst = item & ((1 << kItemInstBits) - 1);
        const int rank = item >> kItemInstBits;
        const l0_problem P = bp.probs[inst];
        const int tsize = bp.team[inst];
        if (bp.timing && rank == 0 && threadIdx.x == 0) {
            int64_t* tim = bp.timing + 8 * static_cast<int64_t>(inst);
            tim[0] = stamp();
            for (int k = 1; k < 6; ++k) tim[k] = 0;
            tim[6] = blockIdx.x;
            tim[7] = tsize;
        }
        solve_dispatch<DLO, DHI>(P, bp, L, inst, rank, tsize);
        if (bp.timing && rank == 0 && threadIdx.x == 0) bp.timing[8 * static_cast<int64_t>(inst) + 1] = stamp();
    }
}

template <int BS, int R = 0>
const void* kernel_for(int range) {
    if constexpr (R >= kBatchRangeCount) {
        return nullptr;
    } else {
        return range == R ? reinterpret_cast<const void*>(&batch_kernel<BS, kBatchRanges[R][0], kBatchRanges[R][1]>)
                          : kernel_for<BS, R + 1>(range);
    }
}

}  // namespace

size_t batch_lds_bytes(int block_threads, int words_cap, int d) {
    const size_t waves = static_cast<size_t>(block_threads / 64);
    return static_cast<size_t>(words_cap) * 4 + waves * 64 * d * 4 + (kBatchQueue + waves * 64) * 4;
}

const void* batch_kernel_fn(int block_threads, int range) {
    switch (block_threads) {
        case 256: return kernel_for<256>(range);
        case 512: return kernel_for<512>(range);
        default: return nullptr;
    }
}

}  // namespace l0
