// Device code of the Parallel-l0 decoder for gfx950.
//
// One solve is a single persistent kernel.  Its workgroups first admit
// themselves as members (the ones running at start-up; the work is split
// among the members only, so the grid barrier never waits for a workgroup
// that could not become resident).  Each iteration of Algorithm 2 runs as
// three phases over all members:
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
// Phases are separated by a barrier over the members built on monotonic
// counters.
#include <hip/hip_runtime.h>

#include <atomic>
#include <climits>
#include <type_traits>

#include "l0_internal.h"
#include "l0_filter.h"
#include "l0_common.h"

static_assert(l0::kRuleL0dec == L0_RULE_L0DEC && l0::kRuleMode == L0_RULE_MODE, "rule codes");

namespace l0 {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int ld_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Which XCD (accelerator complex die) this workgroup runs on, from the
// hardware XCC_ID register.
__device__ __forceinline__ unsigned xcc_id() {
    return static_cast<unsigned>(__builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11))) & 0xFu;
}

// Bounded wait on a monotonic counter with relaxed loads.  Returns false on
// the abort flag or after `limit` wall-clock ticks (then raising the flag).
__device__ __forceinline__ bool wait_at_least(unsigned* p, unsigned target, Ctrl* c, uint64_t limit) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (ld_relaxed(&c->abort)) return false;
        if (wall_clock64() - t0 > limit) {
            __hip_atomic_store(&c->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Where this workgroup sits among the members and for the grid barrier.
struct BarrierSite {
    unsigned member;  // member id: 0 .. count-1
    unsigned count;   // members
    unsigned xcc;     // its XCD
    unsigned nx;      // members on that XCD
    unsigned nxcc;    // XCDs with at least one member
    unsigned epoch;   // barriers passed
    unsigned tl_epochs;  // barriers whose exit the timeline records (its barrier part)
};

constexpr unsigned kClosed = 0x80000000u;  // admission closed (Ctrl::admit)

// Start-up parameters of the solve kernel (wall-clock ticks).
struct Admission {
    uint64_t limit;   // bound of every wait (then the abort flag is raised)
    uint64_t window;  // the first member closes admission this long after its start
    unsigned cap;     // at most this many members
};

// Start-up, in two steps.  admit_register: every workgroup registers on the
// admission word and takes the registration number as its member id; ids
// below min(grid, cap) are members, and a member records its XCD at once
// (during the launch ramp); the member that completes the count publishes
// it.  A member may then do work that needs neither the member count nor
// the other members (the solve's local start) before admit_complete: if
// some workgroups cannot start (the device is shared), the first member
// closes admission `window` ticks after it started, the members being the
// workgroups registered by then (any later one finds admission closed and
// leaves at once); the members wait (relaxed) until all of them have
// recorded their XCDs, and every count is final afterwards.
// admit_register returns 1 for a member and 0 for a workgroup turned away
// (it must leave without touching anything); admit_complete returns 1, or
// -1 when a wait timed out.  With a timeline, member 0 stamps its start in
// entry 0.
struct Registration {
    uint64_t t0;    // start of this workgroup (thread 0)
    unsigned want;  // min(grid, cap)
};

__device__ int admit_register(Ctrl* c, BarrierSite& b, Registration& reg, unsigned cap, int64_t* timeline) {
    __shared__ unsigned s_reg[2];
    if (threadIdx.x == 0) {
        reg.t0 = wall_clock64();
        reg.want = min(gridDim.x, cap);
        const unsigned id = __hip_atomic_fetch_add(&c->admit, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool member = id < reg.want;  // id >= kClosed > want once closed
        unsigned x = 0;
        if (member) {
            if (timeline && id == 0) timeline[0] = static_cast<int64_t>(reg.t0);
            x = xcc_id();
            __hip_atomic_fetch_add(&c->xcount[x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the XCD count is in before the arrival
            __hip_atomic_fetch_add(&c->start, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (id + 1 == reg.want)
                __hip_atomic_store(&c->members, reg.want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_reg[0] = member ? id : kClosed;
        s_reg[1] = x;
    }
    __syncthreads();
    b.member = s_reg[0];
    b.xcc = s_reg[1];
    b.epoch = 0;
    return b.member != kClosed ? 1 : 0;
}

__device__ int admit_complete(Ctrl* c, BarrierSite& b, const Registration& reg, uint64_t window,
                              uint64_t limit) {
    __shared__ unsigned s_site[3];
    __shared__ int s_state;
    if (threadIdx.x == 0) {
        if (b.member == 0 && reg.want > 1) {
            while (__hip_atomic_load(&c->members, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                if (wall_clock64() - reg.t0 > window) {
                    // registrations before the close are ids 0 .. v-1
                    const unsigned v = __hip_atomic_fetch_or(&c->admit, kClosed, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&c->members, min(v & (kClosed - 1u), reg.want), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        int state = wait_at_least(&c->members, 1u, c, limit) ? 1 : -1;
        const unsigned count = __hip_atomic_load(&c->members, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (state == 1) state = wait_at_least(&c->start, count, c, limit) ? 1 : -1;
        unsigned nx = 0, nxcc = 0;
        for (int i = 0; i < kMaxXcc; ++i) {
            const unsigned v = __hip_atomic_load(&c->xcount[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            nxcc += v != 0;
            if (i == static_cast<int>(b.xcc)) nx = v;
        }
        s_site[0] = count;
        s_site[1] = nx;
        s_site[2] = nxcc;
        s_state = state;
    }
    __syncthreads();
    b.count = s_site[0];
    b.nx = s_site[1];
    b.nxcc = s_site[2];
    return s_state;
}

// Grid barrier, hierarchical over XCDs.  Each workgroup drains its own memory
// operations (its stores then sit in its XCD's L2: the vector L1 writes
// through), invalidates its CU's L1 and arrives on its XCD's counter.  The
// last arriver of each XCD writes that L2 back (agent-scope release),
// invalidates it, and arrives on the grid counter; every workgroup then
// polls the grid counter with relaxed loads, which leave the caches alone.
// Why the invalidations may come before the barrier completes: from its
// arrival until the grid counter is complete a workgroup loads no data
// (thread 0 only touches the barrier words, the other threads wait at the
// workgroup barrier), and the XCD's last arriver invalidates the L2 only
// once every workgroup of its XCD has arrived; so no line can enter either
// cache between its invalidation and the completion, which follows every
// XCD's writeback.  Loads after the barrier therefore miss on anything
// written elsewhere and read it from memory.  The L1 invalidation must be
// agent-scope (it also invalidates the L2's non-coherent lines): a
// workgroup-scope one leaves the L1's lines in place here, and decodes went
// wrong with it (16 of 8192 small decodes, once the index loads were cached).
// One hop of waiting, the invalidations off the critical path except the
// last arriver's.  A wait longer than `limit` raises the abort flag and every
// workgroup leaves the kernel.  With a timeline, workgroup 0 stamps the wall
// clock.
__device__ bool grid_sync(Ctrl* c, BarrierSite& b, uint64_t limit, int64_t* timeline = nullptr) {
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this thread's loads and stores are done
    __syncthreads();
    b.epoch += 1;
    if (threadIdx.x == 0) {
        // this CU's L1 (and the L2's non-coherent lines), agent scope; the
        // wait covers the invalidation
        asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
        unsigned* xa = &c->xarrive[b.xcc * kXccStride];
        const unsigned old = __hip_atomic_fetch_add(xa, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == b.epoch * b.nx) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // L2 writeback, waited for
            // the XCD's L2 (and this CU's L1), complete before the arrival
            asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
            __hip_atomic_fetch_add(&c->bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_ok = wait_at_least(&c->bar, b.epoch * b.nxcc, c, limit) ? 1 : 0;
        if (timeline && b.member == 0 && b.epoch < b.tl_epochs)
            timeline[b.epoch] = static_cast<int64_t>(wall_clock64());
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

// Maximum of a double over the workgroup; the result is valid in every thread.
__device__ double block_max(double v) {
    __shared__ double s_part[kWaves];
    __shared__ double s_total;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t = fmax(t, s_part[w]);
        s_total = t;
    }
    __syncthreads();
    return s_total;
}

__device__ __forceinline__ int64_t soa_index(int64_t j, int t, int d) {
    return ((j / kTile) * d + t) * kTile + (j % kTile);
}

// Row index of column j's t-th neighbour in the repacked store (16-bit
// entries when every row fits, else 32-bit).
template <bool ROWS16>
__device__ __forceinline__ int soa_row(const void* soa, int64_t j, int t, int d) {
    if constexpr (ROWS16) return static_cast<const uint16_t*>(soa)[soa_index(j, t, d)];
    else return static_cast<const int32_t*>(soa)[soa_index(j, t, d)];
}

template <int WM>
struct Words {
    static constexpr bool kLds = WM != kWordsGlobal;
    static constexpr bool kRows16 = WM == kWordsLds32 || WM == kWordsLds16;
    using T = typename std::conditional<WM == kWordsLds16, uint16_t,
                                        typename std::conditional<WM == kWordsLds8, uint8_t, uint32_t>::type>::type;
};

// The bucket word of row i in the 32-bit layout, from a word array of mode WM.
template <int WM>
__device__ __forceinline__ uint32_t word_at(const void* words, uint32_t i) {
    using T = typename Words<WM>::T;
    const T w = static_cast<const T*>(words)[i];
    if constexpr (WM == kWordsLds16) return unfold_word(w);
    else if constexpr (WM == kWordsLds8) return unfold_word8(w);
    else return w;
}

// Store row i's bucket word (32-bit layout w) in a word array of mode WM.
template <int WM>
__device__ __forceinline__ void put_word(void* words, uint32_t i, uint32_t w) {
    if constexpr (WM == kWordsLds16) static_cast<uint16_t*>(words)[i] = fold_word(w);
    else if constexpr (WM == kWordsLds8) static_cast<uint8_t*>(words)[i] = fold_word8(w);
    else static_cast<uint32_t*>(words)[i] = w;
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

// The state apply_update and the residual helpers work on (field names as
// theirs expect): the touched-row list is the one of the current
// iteration's parity, so a workgroup still reading the previous iteration's
// list is never overwritten by one that runs ahead.
struct SolveState {
    double* x;
    const double* w;
    const double* y;
    uint32_t* member;
    int32_t* slot_cnt;
    int32_t* slot_sorted;
    int32_t* aff_flag;
    int32_t* aff_list;
    const int32_t* row_off;
    int32_t* slots;
};

__device__ __forceinline__ SolveState state_of(const SolveParams& p, int l) {
    SolveState s;
    s.x = p.x;
    s.w = p.w;
    s.y = p.y;
    s.member = p.member;
    s.slot_cnt = p.slot_cnt;
    s.slot_sorted = p.slot_sorted;
    s.aff_flag = p.aff_flag;
    s.aff_list = p.aff_list + static_cast<int64_t>(l & 1) * p.m;
    s.row_off = p.row_off;
    s.slots = p.slots;
    return s;
}

// ---------------------------------------------------------------------------
// the score of one column (eq. (selection_l0))
// ---------------------------------------------------------------------------

// A workgroup's updates of one vote, gathered in LDS so that the counters
// every workgroup shares (updates, support size, touched-row list length) see
// one atomic per workgroup, not one per update: atomics on one address are
// served one at a time (1361 updates in the first vote at n = 2^20).
// Touched rows wait in `rows` for their list positions; those that do not
// fit are appended at once.
constexpr int kAffBuf = 512;
struct WgUpdates {
    int t;     // updates
    int s;     // columns entering the support
    int a;     // touched rows reserved in `rows` (may pass kAffBuf)
    int base;  // their first position in the touched-row list
    int rows[kAffBuf];
};

// apply_update (l0_common.h) with the shared counters gathered in u: x_hat_j
// += w, the support bit, the per-row support lists and the touched flags as
// there; the count of updates and of new support columns in LDS; touched
// rows into u->rows (the part past kAffBuf straight to the list).
template <int D>
__device__ void apply_update_wg(const SolveState& p, WgUpdates* u, int32_t* affc, int64_t j, double w,
                                const int (&rows)[D]) {
    const double x0 = p.x[j];
    const uint32_t bit = 1u << (j & 31);
    const uint32_t old = __hip_atomic_fetch_or(&p.member[j >> 5], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int first[D], off[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        first[t] = __hip_atomic_exchange(&p.aff_flag[rows[t]], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        off[t] = p.row_off[rows[t]];
    }
    atomicAdd(&u->t, 1);
    const bool fresh = (old & bit) == 0;
    int q[D];
    if (fresh) {
        atomicAdd(&u->s, 1);
#pragma unroll
        for (int t = 0; t < D; ++t) q[t] = fetch_add(&p.slot_cnt[rows[t]], 1);
    }
    int nfirst = 0;
#pragma unroll
    for (int t = 0; t < D; ++t) nfirst += first[t] == 0;
    if (nfirst) {
        const int k = atomicAdd(&u->a, nfirst);
        const int nbuf = k < kAffBuf ? min(nfirst, kAffBuf - k) : 0;
        int qa = nbuf < nfirst ? fetch_add(affc, nfirst - nbuf) : 0;
        int e = 0;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            if (first[t] != 0) continue;
            if (e < nbuf) u->rows[k + e] = rows[t];
            else p.aff_list[qa++] = rows[t];
            ++e;
        }
    }
    if (fresh) {
#pragma unroll
        for (int t = 0; t < D; ++t) p.slots[off[t] + q[t]] = static_cast<int>(j);
    }
    p.x[j] = x0 + w;
}

// Exact scoring of one column that passed the bucket filter: its rows come
// from the repacked index store, its values from the FP64 residual.
// (Shifted rules: the one candidate of this pass, at position pos.)
template <int D, bool ROWS16>
__device__ void score_exact(const SolveParams& p, const SolveState& st, int l, int64_t j, double tau, int pos,
                            WgUpdates* u) {
    int rows[D];
#pragma unroll
    for (int t = 0; t < D; ++t) rows[t] = soa_row<ROWS16>(p.soa, j, t, D);
    double v[D];
#pragma unroll
    for (int t = 0; t < D; ++t) v[t] = p.r[rows[t]];
    double om;
    const bool sel = rule_is_shifted(p.rule) ? exact_score_shifted<D>(v, pos, tau, p.rule, p.a, om)
                                             : exact_score<D>(v, tau, p.rule, p.a, om);
    if (sel) apply_update_wg<D>(st, u, &p.affc[l], j, column_update(st, j, om), rows);
}

constexpr int kQueue = 2048;  // per-workgroup queue of columns passing the filter

// A chunk is the unit a wave streams: 128 columns (two 16-bit rows per lane
// and plane) for 16-bit rows, else 64 columns (one 32-bit row per lane).
// Each neighbour plane of a chunk is one coalesced 256-byte load.
template <bool ROWS16>
struct Chunk {
    static constexpr uint32_t kCols = ROWS16 ? 128 : 64;
    static constexpr uint32_t kPerTile = kTile / kCols;
};

// Index loads of the vote's stream: streaming (nt) loads, or ordinary cached
// loads when the index store is small enough to stay in the caches between
// votes.  Measured per solve, nt against cached: n = 2^24 (235 MB store)
// 181 vs 196 us, 2^23 (117 MB) 86.0 vs 86.5, 2^22 (59 MB) 82.4 vs 83.9,
// 2^20 (29 MB, 32-bit rows) 190.5 vs 188.5.
constexpr uint64_t kStreamNtBytes = 48ull << 20;

template <int D, bool ROWS16, bool NT = true>
__device__ __forceinline__ void load_chunk(const void* soa, uint32_t g, uint32_t lane, uint32_t (&rows)[D]) {
    constexpr uint32_t plane = ROWS16 ? kTile / 2 : kTile;  // 32-bit words per plane of a tile
    constexpr uint32_t per = Chunk<ROWS16>::kPerTile;
    // one base address; the planes are immediate offsets from it
    const uint32_t* __restrict__ q = static_cast<const uint32_t*>(soa) +
                                     (static_cast<uint64_t>(g / per) * (D * plane) + (g % per) * 64u + lane);
#pragma unroll
    for (int t = 0; t < D; ++t) {
        if constexpr (NT) rows[t] = __builtin_nontemporal_load(q + t * plane);
        else rows[t] = q[t * plane];
    }
}

// Filter the columns of one chunk (half a chunk for 16-bit rows) and append
// the passing ones to the workgroup's LDS queue.  Only LDS is written here:
// once the queue is full, positions are clamped to its last slot and the
// overflow flag is raised (the queue is then discarded and the workgroup's
// chunks are filtered again, see vote_score).
template <int D>
__device__ __forceinline__ void filter_and_queue(const SolveParams& p, const uint32_t (&w)[D], uint32_t j,
                                                 uint32_t n, uint32_t lane, int* q_items, int* q_count,
                                                 int* q_ovf) {
    const bool pass = bucket_filter<D>(w, p.a, p.rule) && j < n;
    const unsigned long long mask = __ballot(pass);
    if (mask) {
        int base = 0;
        if (lane == 0) base = atomicAdd(q_count, __popcll(mask));
        base = __shfl(base, 0);
        const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (pass) q_items[pos < kQueue ? pos : kQueue - 1] = static_cast<int>(j);
        if (lane == 0 && base + __popcll(mask) > kQueue) *q_ovf = 1;
    }
}

// The rows of half h of a chunk's lane (16-bit rows: two per 32-bit word).
template <bool ROWS16>
__device__ __forceinline__ uint32_t chunk_row(uint32_t r, int h) {
    if constexpr (ROWS16) return h ? (r >> 16) : (r & 0xFFFFu);
    else return r;
}

// Filter one chunk whose row indices are in `rows`; `words` is the LDS copy
// of the bucket words (or the global array for kWordsGlobal).
template <int D, int WM>
__device__ __forceinline__ void filter_chunk(const SolveParams& p, const void* words, const uint32_t (&rows)[D],
                                             uint32_t g, uint32_t n, uint32_t lane, int* q_items, int* q_count,
                                             int* q_ovf) {
    constexpr bool R16 = Words<WM>::kRows16;
#pragma unroll
    for (int h = 0; h < (R16 ? 2 : 1); ++h) {
        uint32_t w[D];
#pragma unroll
        for (int t = 0; t < D; ++t) w[t] = word_at<WM>(words, chunk_row<R16>(rows[t], h));
        const uint32_t j = R16 ? g * Chunk<true>::kCols + 2 * lane + h : g * Chunk<false>::kCols + lane;
        filter_and_queue<D>(p, w, j, n, lane, q_items, q_count, q_ovf);
    }
}

// Vote, first half.  Each wave streams its chunks (g = wave, wave + stride,
// ...) with two chunks' row indices in flight (two register buffers taking
// turns, so no copy waits on a load), gathers the rows' bucket words, runs
// the bucket filter and queues the passing columns in LDS.  It loads nothing
// but the index store and stores nothing to global memory, so every wait
// covers loads only.  Chunks are assigned statically: handing them out
// through atomic counters costs more than the imbalance it removes (a wave
// cannot wait for a chunk's loads without also waiting for an older claim).
// l: the iteration (timeline).
template <int D, int WM, bool NT>
__device__ void vote_stream(const SolveParams& p, int l, const void* lds_w, int* q_items, int* q_count,
                            int* q_ovf, unsigned member, unsigned members) {
    constexpr bool R16 = Words<WM>::kRows16;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nchunks = static_cast<uint32_t>(p.ntiles) * Chunk<R16>::kPerTile;
    const uint32_t n = static_cast<uint32_t>(p.n);
    const void* words = Words<WM>::kLds ? lds_w : p.rword;
    // chunk numbers are uniform over the wave (scalar registers)
    const uint32_t stride = __builtin_amdgcn_readfirstlane(members * kWaves);
    const uint32_t first = __builtin_amdgcn_readfirstlane(member * kWaves + (threadIdx.x >> 6));
    // prefetches past the last chunk read the last chunk again (an L2 hit;
    // unconditional loads keep the waits exact)
    const uint32_t last = nchunks - 1;
    uint32_t g = first;
    uint32_t a[D], b[D];
    load_chunk<D, R16, NT>(p.soa, min(g, last), lane, a);
    load_chunk<D, R16, NT>(p.soa, min(g + stride, last), lane, b);
    while (g < nchunks) {
        filter_chunk<D, WM>(p, words, a, g, n, lane, q_items, q_count, q_ovf);
        load_chunk<D, R16, NT>(p.soa, min(g + 2 * stride, last), lane, a);
        g += stride;
        if (g >= nchunks) break;
        filter_chunk<D, WM>(p, words, b, g, n, lane, q_items, q_count, q_ovf);
        load_chunk<D, R16, NT>(p.soa, min(g + 2 * stride, last), lane, b);
        g += stride;
    }
    __syncthreads();
    if (p.timeline && member == 0 && threadIdx.x == 0)
        p.timeline[3 * p.max_iter + 9 + 3 * l] = static_cast<int64_t>(wall_clock64());
}

// The exact scoring of the columns the workgroup's stream queued (see
// vote_stream), or, if its queue overflowed, of every passing column of its
// chunks, filtered again.
template <int D, int WM>
__device__ void vote_score(const SolveParams& p, const SolveState& st, int l, double tau, const void* lds_w,
                           int* q_items, int* q_count, int* q_ovf, int pos, unsigned member, unsigned members,
                           WgUpdates* u) {
    constexpr bool R16 = Words<WM>::kRows16;
    if (*q_ovf == 0) {
        const int cnt = *q_count;
        for (int q = threadIdx.x; q < cnt; q += kBlock) score_exact<D, R16>(p, st, l, q_items[q], tau, pos, u);
    } else {
        // overflow: every chunk of this wave again, passing columns scored directly
        constexpr uint32_t kCols = Chunk<R16>::kCols;
        const uint32_t lane = threadIdx.x & 63;
        const uint32_t nchunks = static_cast<uint32_t>(p.ntiles) * Chunk<R16>::kPerTile;
        const uint32_t n = static_cast<uint32_t>(p.n);
        const void* words = Words<WM>::kLds ? lds_w : p.rword;
        const uint32_t stride = __builtin_amdgcn_readfirstlane(members * kWaves);
        const uint32_t first = __builtin_amdgcn_readfirstlane(member * kWaves + (threadIdx.x >> 6));
        for (uint32_t c = first; c < nchunks; c += stride) {
            uint32_t rows[D];
            load_chunk<D, R16>(p.soa, c, lane, rows);
#pragma unroll
            for (int h = 0; h < (R16 ? 2 : 1); ++h) {
                uint32_t w[D];
#pragma unroll
                for (int t = 0; t < D; ++t) w[t] = word_at<WM>(words, chunk_row<R16>(rows[t], h));
                const uint32_t j = c * kCols + (R16 ? 2 * lane + h : lane);
                if (bucket_filter<D>(w, p.a, p.rule) && j < n) score_exact<D, R16>(p, st, l, j, tau, pos, u);
            }
        }
    }
    __syncthreads();
    // the workgroup's shares of the shared counters, one atomic each, and
    // the positions of its buffered touched rows
    const int nbuf = min(u->a, kAffBuf);
    if (threadIdx.x == 0) {
        if (u->t) fetch_add(&p.tcount[l], u->t);
        if (u->s) fetch_add(&p.ctrl->support, u->s);
        u->base = nbuf ? fetch_add(&p.affc[l], nbuf) : 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nbuf; t += kBlock) st.aff_list[u->base + t] = u->rows[t];
    __syncthreads();
    if (threadIdx.x == 0) {
        *q_count = 0;
        *q_ovf = 0;
        u->t = u->s = u->a = 0;
        if (p.timeline && member == 0)
            p.timeline[3 * p.max_iter + 10 + 3 * l] = static_cast<int64_t>(wall_clock64());
    }
}

// Copy the global bucket words (mode WM, m of them) into this workgroup's
// LDS copy: 16-byte loads, four in flight per thread, the tail word by word.
template <int WM>
__device__ void stage_words(const SolveParams& p, void* lds_w) {
    using T = typename Words<WM>::T;
    const int bytes = p.m * static_cast<int>(sizeof(T));
    const int n16 = bytes >> 4;
    const uint4* src4 = static_cast<const uint4*>(p.rword);
    uint4* dst4 = static_cast<uint4*>(lds_w);
    const int tid = threadIdx.x;
    int i = tid;
    for (; i + 3 * kBlock < n16; i += 4 * kBlock) {
        const uint4 a0 = src4[i], a1 = src4[i + kBlock];
        const uint4 a2 = src4[i + 2 * kBlock], a3 = src4[i + 3 * kBlock];
        dst4[i] = a0;
        dst4[i + kBlock] = a1;
        dst4[i + 2 * kBlock] = a2;
        dst4[i + 3 * kBlock] = a3;
    }
    for (; i < n16; i += kBlock) dst4[i] = src4[i];
    const T* src = static_cast<const T*>(p.rword);
    T* dst = static_cast<T*>(lds_w);
    for (int t = ((n16 << 4) / static_cast<int>(sizeof(T))) + tid; t < p.m; t += kBlock) dst[t] = src[t];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// the persistent solve kernel
// ---------------------------------------------------------------------------

// Residual rows whose support-list merge is long for one thread (the
// insertion of the new entries into the sorted prefix moves about
// new x count entries of global memory one at a time) go to the whole
// workgroup, at most kHeavyRows per workgroup and pass; lists up to half the
// queue's LDS.
constexpr int kHeavyRows = 32;
constexpr int kHeavyWork = 256;

template <class S>
__device__ __forceinline__ bool heavy_row(const S& st, int i) {
    const int cnt = st.slot_cnt[i];
    const int fresh = cnt - st.slot_sorted[i];
    return cnt <= kQueue / 2 && fresh > 0 && fresh * cnt > kHeavyWork;
}

// row_residual for one row, by the whole workgroup (every thread calls it;
// the result is valid in thread 0), buf: kQueue ints of LDS.  The list's
// column ids are distinct, so entry v goes to position (entries below v):
// one thread per entry counts them; the sorted list is written back; the
// column terms are gathered 512 at a time into LDS and thread 0 adds them in
// ascending j from +0.0 (the order and rounding of row_residual).
template <class S>
__device__ double wg_row_residual(const S& st, int i, int* buf) {
    const int tid = threadIdx.x;
    const int cnt = st.slot_cnt[i];
    int* const list = st.slots + st.row_off[i];
    int* const a = buf;
    int* const b = buf + kQueue / 2;
    for (int t = tid; t < cnt; t += kBlock) a[t] = list[t];
    __syncthreads();
    for (int t = tid; t < cnt; t += kBlock) {
        const int v = a[t];
        int below = 0;
        for (int u = 0; u < cnt; ++u) below += a[u] < v;
        b[below] = v;
    }
    __syncthreads();
    for (int t = tid; t < cnt; t += kBlock) list[t] = b[t];
    if (tid == 0) st.slot_sorted[i] = cnt;
    double* const terms = reinterpret_cast<double*>(a);  // kQueue / 4 doubles
    constexpr int kChunk = kQueue / 4;
    double sum = 0.0;
    for (int c0 = 0; c0 < cnt; c0 += kChunk) {
        const int len = min(kChunk, cnt - c0);
        for (int t = tid; t < len; t += kBlock) terms[t] = column_term(st, b[c0 + t]);
        __syncthreads();
        if (tid == 0)
            for (int t = 0; t < len; ++t) sum += terms[t];
        __syncthreads();
    }
    return st.y[i] - sum;
}

// The new residual value rn of touched row i: r_i, its bucket word and its
// touched flag; returns the change of ||r||_0.
template <int WM>
__device__ __forceinline__ int finish_row(const SolveParams& p, int i, double rn, double tau, double inv_w) {
    const bool was = fabs(p.r[i]) > tau;
    const bool now = fabs(rn) > tau;
    p.r[i] = rn;
    put_word<WM>(p.rword, static_cast<uint32_t>(i), row_word(rn, tau, inv_w));
    p.aff_flag[i] = 0;
    return static_cast<int>(now) - static_cast<int>(was);
}

// x_hat = 0, this member's share: the members split x_hat into contiguous
// runs written by plain 16-byte stores (a double before the first 16-byte
// boundary and an odd last one apart; an x not 8-byte aligned by plain
// 8-byte stores).  Measured in the n = 2^24 solve, against the same stores
// striding over the grid and against streaming (nt) stores either way, this
// form was the fastest by 2-10 us: the dirty lines it leaves in L2 drain
// under the first vote.  Nothing here waits for the stores.
__device__ void clear_x_share(double* x, int64_t n, unsigned member, unsigned count) {
    typedef double double2v __attribute__((ext_vector_type(2)));
    const uintptr_t addr = reinterpret_cast<uintptr_t>(x);
    if (addr & 7) {
        const int64_t per = (n + count - 1) / count;
        const int64_t j0 = per * member, j1 = min(j0 + per, n);
        for (int64_t j = j0 + threadIdx.x; j < j1; j += kBlock) x[j] = 0.0;
        return;
    }
    const int64_t head = (addr & 15) && n > 0 ? 1 : 0;
    const int64_t pairs = (n - head) / 2;
    const int64_t per = (pairs + count - 1) / count;
    const int64_t q0 = per * member, q1 = min(q0 + per, pairs);
    double2v* xp = reinterpret_cast<double2v*>(x + head);
    const double2v z = {0.0, 0.0};
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock) xp[q] = z;
    if (member == 0 && threadIdx.x == 0) {
        if (head) x[0] = 0.0;
        if ((n - head) & 1) x[n - 1] = 0.0;
    }
}

// Waves per SIMD the compiler must allow: one resident workgroup per CU (4
// waves), which leaves 128 VGPRs per lane (no spills).  Two workgroups per CU
// (8 waves, 64 VGPRs) were measured slower: the second workgroup on a CU
// streamed its share about a third slower than the first, and every pass
// waited for it.
template <int D>
struct Occ {
    static constexpr int kWavesPerEU = 4;
};

template <int D, int WM>
__global__ void __launch_bounds__(kBlock, Occ<D>::kWavesPerEU) solve_kernel(SolveParams p, Admission adm) {
    extern __shared__ uint32_t lds_w[];
    __shared__ int q_items[kQueue];
    __shared__ int q_count, q_ovf;
    __shared__ int h_rows[kHeavyRows];
    __shared__ int h_count;
    __shared__ WgUpdates wg_upd;
    constexpr bool R16 = Words<WM>::kRows16;
    if (threadIdx.x == 0) {
        q_count = q_ovf = 0;
        wg_upd.t = wg_upd.s = wg_upd.a = 0;
    }
    const int tid = threadIdx.x;
    Ctrl* c = p.ctrl;
    const uint64_t limit = adm.limit;
    BarrierSite site;
    Registration reg;
    if (!admit_register(c, site, reg, adm.cap, p.timeline)) return;  // turned away: the members do the work
    // the timeline's barrier part: entries 1 .. 3*max_iter + 6 (a shifted
    // rule's empty passes can pass more barriers; those are not recorded)
    site.tl_epochs = 3 * static_cast<unsigned>(p.max_iter) + 7;

    // Without a resume vector and with 32-bit words in LDS (y then has at
    // most 36864 entries), every workgroup derives max |y|, tau, ||y||_0 and
    // all bucket words of r = y from y itself (it needs no other member): no
    // grid barrier is needed between the start-up and the first vote, and
    // the first pass stages nothing.
    const bool local_init = WM == kWordsLds32 && p.x_init == nullptr;

    // with local_init every y value this thread needs sits in registers:
    // m <= 36864 = kLocalRows * kBlock, loaded once (one memory latency, not
    // one per pass)
    constexpr int kLocalRows = 36;
    static_assert(kLocalRows * kBlock * 4 >= kLdsWordBytes, "local start covers every 32-bit LDS word mode");
    double yv[kLocalRows];
    double ymax = 0.0;
    int nnz = 0;
    if (local_init) {
        // max |y| over every row, in every workgroup (a maximum is exact in
        // any order, so all workgroups agree), during the launch ramp;
        // non-finite y is reported by the shares below
#pragma unroll
        for (int u = 0; u < kLocalRows; ++u)
            if (u * kBlock < p.m) yv[u] = p.y[min(u * kBlock + tid, p.m - 1)];
        double lmax = 0.0;
#pragma unroll
        for (int u = 0; u < kLocalRows; ++u)
            if (u * kBlock < p.m && isfinite(yv[u])) lmax = fmax(lmax, fabs(yv[u]));
        ymax = block_max(lmax);
    }

    // the member count and the barrier sites; work is split by member id
    const int state = admit_complete(c, site, reg, adm.window, limit);
    const int64_t gtid = static_cast<int64_t>(site.member) * kBlock + tid;
    const int64_t gsize = static_cast<int64_t>(site.count) * kBlock;
    if (state < 0) {
        if (gtid == 0) write_result(p, 0, L0_DEV_ABORTED, 0, 0, 0);
        return;
    }
    if (p.timeline && site.member == 0 && tid == 0)
        p.timeline[3 * p.max_iter + 7] = static_cast<int64_t>(wall_clock64());
    // x_hat = 0 for a solve from zero, a pure write stream: issued before
    // the word arithmetic below, which loads nothing, so the stores drain
    // under it (mixed with the first vote's index stream they cost more
    // than alone)
    if (p.x_init == nullptr) clear_x_share(p.x, p.n, site.member, site.count);
    const double tau0 = (p.tol_mode == L0_TOL_RELATIVE) ? p.tol * ymax : p.tol;
    if (local_init) {
        // ||y||_0 and the bucket words of r = y, all of them into LDS
        const double iw = 1.0 / bucket_width(tau0, ymax);
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < kLocalRows; ++u) {
            const int i = u * kBlock + tid;
            if (u * kBlock < p.m && i < p.m) {
                lds_w[i] = row_word(yv[u], tau0, iw);
                cnt += fabs(yv[u]) > tau0;
            }
        }
        nnz = block_sum(cnt);
        // this workgroup's share of the words to the global word array
        for (int64_t i = gtid; i < p.m; i += gsize) static_cast<uint32_t*>(p.rword)[i] = lds_w[i];
        if (gtid == 0) __hip_atomic_store(&c->nnz, nnz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // --- init: x_hat of a resume (copied from x_init), support bitmap,
    //     per-row state, max |y|, finiteness of y, usable column weights
    {
        int bad_w = 0;
        if (p.x_init)
            for (int64_t j = gtid; j < p.n; j += gsize) p.x[j] = p.x_init[j];
        if (p.w)
            for (int64_t j = gtid; j < p.n; j += gsize)
                if (!weight_ok(p.w[j])) bad_w = 1;
        if (wave_count(bad_w != 0) && (tid & 63) == 0) atomicOr(&c->err, kErrBadWeight);
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
            if (local_init) p.r[i] = yi;
        }
        if (!local_init) {
            // one atomic per workgroup (atomics on one address are served
            // one at a time)
            lmax = block_max(lmax);
            if (tid == 0 && lmax > 0.0)
                atomicMax(reinterpret_cast<unsigned long long*>(&c->maxabs_bits),
                          static_cast<unsigned long long>(__double_as_longlong(lmax)));
        }
        if (wave_count(bad != 0) && (tid & 63) == 0) atomicOr(&c->err, kErrNonfiniteY);
        if (gtid == 0) {
            const int mb = *p.bad_input;
            if (mb) atomicOr(&c->err, mb);
        }
    }
    if (!grid_sync(c, site, limit, p.timeline)) {
        if (gtid == 0) write_result(p, 0, L0_DEV_ABORTED, 0, 0, 0);
        return;
    }
    const int err = ld_relaxed(&c->err);
    if (err) {
        // x_hat is zero already
        if (gtid == 0) write_result(p, 0, error_outcome(err), 0, 0, 0);
        return;
    }
    if (!local_init)
        ymax = __longlong_as_double(static_cast<long long>(
            __hip_atomic_load(&c->maxabs_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    const double tau = (p.tol_mode == L0_TOL_RELATIVE) ? p.tol * ymax : p.tol;
    const double inv_w = 1.0 / bucket_width(tau, ymax);

    // --- resume: enter the nonzeros of x_init into the support lists
    if (p.x_init) {
        for (int64_t j = gtid; j < p.n; j += gsize) {
            if (p.x[j] == 0.0) continue;
            atomicOr(&p.member[j >> 5], 1u << (j & 31));
            atomicAdd(&c->support, 1);
            for (int t = 0; t < D; ++t) {
                const int i = soa_row<R16>(p.soa, j, t, D);
                const int q = atomicAdd(&p.slot_cnt[i], 1);
                p.slots[p.row_off[i] + q] = static_cast<int>(j);
            }
        }
        if (!grid_sync(c, site, limit, p.timeline)) {
            if (gtid == 0) write_result(p, 0, L0_DEV_ABORTED, 0, 0, 0);
            return;
        }
    }

    // --- r = y - A x_hat and ||r||_0 (done above in the local start)
    if (!local_init) {
        const SolveState st0 = state_of(p, 0);
        int wnz = 0;
        for (int64_t i = gtid; i < p.m; i += gsize) {
            const double ri = p.x_init ? row_residual(st0, static_cast<int>(i)) : p.y[i];
            p.r[i] = ri;
            put_word<WM>(p.rword, static_cast<uint32_t>(i), row_word(ri, tau, inv_w));
            wnz += wave_count(fabs(ri) > tau);
        }
        const int b = block_sum((tid & 63) == 0 ? wnz : 0);
        if (tid == 0 && b) atomicAdd(&c->nnz, b);
        if (!grid_sync(c, site, limit, p.timeline)) {
            if (gtid == 0) write_result(p, 0, L0_DEV_ABORTED, 0, 0, 0);
            return;
        }
        nnz = ld_relaxed(&c->nnz);
        // every bucket word into this workgroup's LDS copy, once: after each
        // iteration only the rows it touched are refreshed
        if (Words<WM>::kLds) stage_words<WM>(p, lds_w);
    }
    if (gtid == 0 && p.trace) p.trace[0] = nnz;

    // Vote passes are counted apart from iterations: a shifted rule's pass
    // that selects nothing is followed by another (the next position) and
    // the run stalls after D such passes in a row.
    int l = 0, pass = 0, empty = 0;
    const bool shifted = rule_is_shifted(p.rule);
    const bool stream_nt = static_cast<uint64_t>(p.ntiles) * D * kTile * (R16 ? 2 : 4) > kStreamNtBytes;
    int outcome;
    long long updates = 0;
    for (;;) {
        if (nnz == 0 || l == p.max_iter) {
            outcome = nnz == 0 ? L0_CONVERGED : L0_MAX_ITER;
            break;
        }
        const int pos = pass % D;
        const SolveState st = state_of(p, l);

        // vote on the same residual for every column (the LDS copy of the
        // words is current: staged at the start, refreshed after each
        // iteration)
        if (p.timeline && site.member == 0 && tid == 0)
            p.timeline[3 * p.max_iter + 8 + 3 * l] = static_cast<int64_t>(wall_clock64());
        if (stream_nt) vote_stream<D, WM, true>(p, l, lds_w, q_items, &q_count, &q_ovf, site.member, site.count);
        else vote_stream<D, WM, false>(p, l, lds_w, q_items, &q_count, &q_ovf, site.member, site.count);
        vote_score<D, WM>(p, st, l, tau, lds_w, q_items, &q_count, &q_ovf, pos, site.member, site.count,
                          &wg_upd);
        if (!grid_sync(c, site, limit, p.timeline)) {
            if (gtid == 0) write_result(p, l, L0_DEV_ABORTED, nnz, 0, updates);
            return;
        }
        ++pass;
        const int tc = ld_relaxed(&p.tcount[l]);
        if (tc == 0) {
            if (shifted && ++empty < D) continue;
            outcome = L0_STALLED;
            break;
        }
        empty = 0;

        // residual update of the touched rows, ||r||_0 by its change; a row
        // whose list merge would be long for one thread is handed to the
        // whole workgroup (the queue's LDS is free here)
        const int na = ld_relaxed(&p.affc[l]);
        {
            if (tid == 0) h_count = 0;
            __syncthreads();
            int delta = 0;
            // touched rows dealt round-robin over the workgroups (entry q to
            // workgroup q mod count), so that a short list occupies every CU's
            // memory pipeline instead of the first few workgroups'
            for (int64_t q = static_cast<int64_t>(tid) * site.count + site.member; q < na; q += gsize) {
                const int i = st.aff_list[q];
                if (heavy_row(st, i)) {
                    const int h = atomicAdd(&h_count, 1);
                    if (h < kHeavyRows) {
                        h_rows[h] = i;
                        continue;
                    }
                }
                delta += finish_row<WM>(p, i, row_residual(st, i), tau, inv_w);
            }
            __syncthreads();
            const int nh = min(h_count, kHeavyRows);
            for (int h = 0; h < nh; ++h) {
                const int i = h_rows[h];
                const double rn = wg_row_residual(st, i, q_items);
                if (tid == 0) delta += finish_row<WM>(p, i, rn, tau, inv_w);
            }
            const int b = block_sum(delta);
            if (tid == 0 && b) atomicAdd(&c->nnz, b);
        }
        if (!grid_sync(c, site, limit, p.timeline)) {
            if (gtid == 0) write_result(p, l, L0_DEV_ABORTED, nnz, 0, updates);
            return;
        }
        nnz = ld_relaxed(&c->nnz);
        updates += tc;
        // refresh this workgroup's LDS words of the rows the iteration
        // touched (the list of this iteration's parity: the next iteration
        // appends to the other one)
        if (Words<WM>::kLds) {
            using T = typename Words<WM>::T;
            if (static_cast<int64_t>(na) * 64 > static_cast<int64_t>(p.m) * static_cast<int64_t>(sizeof(T))) {
                // many rows: a 64-byte line per scattered word costs more
                // than copying every word again
                stage_words<WM>(p, lds_w);
            } else {
                T* lw = reinterpret_cast<T*>(lds_w);
                const T* gw = static_cast<const T*>(p.rword);
                for (int q = tid; q < na; q += kBlock) {
                    const int i = st.aff_list[q];
                    lw[i] = gw[i];
                }
                __syncthreads();
            }
        }
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

// Repack col_idx (each column's d rows contiguous) into the tiled neighbour
// planes, check every row index and that no column lists a row twice, and
// count row degrees (LDS histogram when m
// fits, else global atomics).  A group is 64 columns: their 64*D contiguous
// indices arrive by D coalesced loads, go through the wave's LDS staging area
// and leave as D contiguous 64-entry runs, one per neighbour plane.  Each wave
// issues the loads of RepackGroups<D> consecutive groups before it stages the
// first, so enough reads are in flight to stream at HBM rate; groups that lie
// wholly inside the array are read from one base address (immediate offsets,
// few address registers), only the last, partial one index by index.
template <int D>
struct RepackGroups {
    static constexpr int value = D >= 28 ? 1 : 28 / D;
};

template <int D, typename IT, bool LDS_HIST>
__global__ void __launch_bounds__(1024) repack_kernel(const int32_t* col_idx, MatrixView A) {
    constexpr int G = RepackGroups<D>::value;
    extern __shared__ int sh[];
    int* hist = sh;
    int* stage = sh + (LDS_HIST ? A.m : 0) + (threadIdx.x >> 6) * (64 * D);
    const int lane = threadIdx.x & 63;
    if (LDS_HIST)
        for (int i = threadIdx.x; i < A.m; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int64_t nd = A.n * D;
    const int64_t ngroups = A.ntiles * (kTile / 64);
    // the wave index is uniform across the wave: a scalar loop (no exec mask,
    // scalar addresses)
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * kRepackWaves +
                         __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRepackWaves * G;
    const unsigned m = static_cast<unsigned>(A.m);
    int bad = 0;
    for (int64_t g0 = wave * G; g0 < ngroups; g0 += stride) {
        int v[G][D];
        if ((g0 + G) * 64 * D <= nd) {
            const int32_t* base = col_idx + g0 * 64 * D + lane;
#pragma unroll
            for (int gi = 0; gi < G; ++gi)
#pragma unroll
                for (int k = 0; k < D; ++k) v[gi][k] = __builtin_nontemporal_load(base + (gi * D + k) * 64);
        } else {
            // indices past the end read the last entry; their rows become 0
#pragma unroll
            for (int gi = 0; gi < G; ++gi)
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const int64_t e = (g0 + gi) * 64 * D + k * 64 + lane;
                    v[gi][k] = e < nd ? __builtin_nontemporal_load(&col_idx[e]) : 0;
                }
        }
#pragma unroll
        for (int gi = 0; gi < G; ++gi) {
            const int64_t g = g0 + gi;
            if (g >= ngroups) continue;  // uniform across the wave
            const int64_t e0 = g * 64 * D + lane;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int row = v[gi][k];
                const bool inside = e0 + k * 64 < nd;
                const bool ok = static_cast<unsigned>(row) < m;
                if (inside && !ok) bad |= kErrBadIndex;
                if (LDS_HIST && inside && ok) atomicAdd(&hist[row], 1);
                stage[k * 64 + lane] = inside && ok ? row : 0;
            }
            // the wave's LDS stores complete (lgkmcnt(0)) before any lane reads
            // another lane's entries; the wave barrier keeps the compiler from
            // moving the reads above
            __builtin_amdgcn_s_waitcnt(0xC07F);
            __builtin_amdgcn_wave_barrier();
            const int64_t tile = g / (kTile / 64);
            const int c = static_cast<int>(g % (kTile / 64)) * 64 + lane;
            int rr[D];
#pragma unroll
            for (int t = 0; t < D; ++t) rr[t] = stage[lane * D + t];
            // column g*64 + lane lists a row twice (columns past n hold only
            // zeros and are not checked)
            if (g * 64 + lane < A.n && has_repeat<D>(rr)) bad |= kErrRepeatedRow;
            IT out[D];
#pragma unroll
            for (int t = 0; t < D; ++t) out[t] = static_cast<IT>(rr[t]);
            // every lane has read its entries before the next group's stores
            __builtin_amdgcn_s_waitcnt(0xC07F);
            __builtin_amdgcn_wave_barrier();
            IT* dst = static_cast<IT*>(A.soa) + tile * D * kTile + c;
#pragma unroll
            for (int t = 0; t < D; ++t) dst[t * kTile] = out[t];
        }
    }
    if (bad) atomicOr(A.bad_input, bad);
    if (LDS_HIST) {
        __syncthreads();
        for (int i = threadIdx.x; i < A.m; i += blockDim.x)
            if (hist[i]) atomicAdd(&A.deg[i], hist[i]);
    }
}

// Partial degree counts (matrices whose m counts do not fit in the repack
// kernel's LDS): workgroup s counts the rows of its slice of the flat index
// array in LDS, kDegRange rows per pass (the slice is read once per pass,
// mostly from L2 after the first), and stores the counts densely at
// partial[s*m + row].  Indices outside [0, m) are skipped (the repack flags
// them).
__global__ void __launch_bounds__(1024) deg_partial_kernel(const int32_t* col_idx, MatrixView A, int64_t nd) {
    // workgroup (x, y): slice x of the index array, rows y*kDegRange ..
    extern __shared__ int hist[];
    constexpr int U = 16;  // independent loads in flight per thread
    const int tid = threadIdx.x;
    const int64_t lo_e = nd * blockIdx.x / gridDim.x, hi_e = nd * (blockIdx.x + 1) / gridDim.x;
    const int r0 = static_cast<int>(blockIdx.y) * kDegRange;
    const int len = min(kDegRange, A.m - r0);
    for (int i = tid; i < len; i += 1024) hist[i] = 0;
    __syncthreads();
    for (int64_t base = lo_e; base < hi_e; base += int64_t(1024) * U) {
        int v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = base + static_cast<int64_t>(u) * 1024 + tid;
            v[u] = col_idx[e < hi_e ? e : hi_e - 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = base + static_cast<int64_t>(u) * 1024 + tid;
            const unsigned rel = static_cast<unsigned>(v[u] - r0);
            if (e < hi_e && rel < static_cast<unsigned>(len)) atomicAdd(&hist[rel], 1);
        }
    }
    __syncthreads();
    int32_t* part = A.partial + static_cast<int64_t>(blockIdx.x) * A.m + r0;
    for (int i = tid; i < len; i += 1024) part[i] = hist[i];
}

// Sum of an int over a 1024-thread workgroup (valid in every thread).
__device__ int block1024_sum(int v, int* s_wave) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += s_wave[w];
    return t;
}

// deg[i] = sum over the slices of partial[s*m + i], 1024 rows per workgroup,
// and the workgroup's total in blk[blockIdx.x].
__global__ void __launch_bounds__(1024) deg_reduce_kernel(MatrixView A) {
    __shared__ int s_wave[16];
    constexpr int U = 8;  // partial counts in flight per thread
    const int i = blockIdx.x * 1024 + threadIdx.x;
    const int ic = i < A.m ? i : A.m - 1;
    int sum = 0;
    for (int k0 = 0; k0 < A.slices; k0 += U) {
        int v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u < A.slices ? k0 + u : A.slices - 1;
            v[u] = A.partial[static_cast<int64_t>(k) * A.m + ic];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) sum += k0 + u < A.slices ? v[u] : 0;
    }
    if (i < A.m) A.deg[i] = sum;
    const int t = block1024_sum(i < A.m ? sum : 0, s_wave);
    if (threadIdx.x == 0) A.blk[blockIdx.x] = t;
}

// row_off from the degrees and the workgroup totals of deg_reduce_kernel:
// workgroup b adds the totals of the workgroups before it to the exclusive
// scan of its 1024 degrees; the last one also writes row_off[m].  Workgroup
// 0 first clears a one-shot decode's solve control block.
__global__ void __launch_bounds__(1024) scan_blocks_kernel(MatrixView A, int32_t* clear, int64_t clear_count) {
    __shared__ int s_wave[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (blockIdx.x == 0)
        for (int64_t i = tid; i < clear_count; i += 1024) clear[i] = 0;
    const int nblk = static_cast<int>(gridDim.x);
    int before = 0;
    for (int b0 = 0; b0 < static_cast<int>(blockIdx.x); b0 += 1024)
        before += b0 + tid < static_cast<int>(blockIdx.x) ? A.blk[b0 + tid] : 0;
    const int offset = block1024_sum(before, s_wave);
    const int i = blockIdx.x * 1024 + tid;
    const int v = i < A.m ? A.deg[i] : 0;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    __syncthreads();  // s_wave is reused
    if (lane == 63) s_wave[wid] = incl;
    __syncthreads();
    int run = offset + incl - v;
    int total = offset;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        run += w < wid ? s_wave[w] : 0;
        total += s_wave[w];
    }
    if (i < A.m) A.row_off[i] = run;
    if (blockIdx.x == nblk - 1 && tid == 0) A.row_off[A.m] = total;
}

// row_off = exclusive prefix sum of the row degrees (one workgroup), chunk by
// chunk of kScanChunk rows staged in LDS: coalesced loads (kScanPer in flight
// per thread), each thread scans kScanPer consecutive staged entries, the
// workgroup scans the thread sums, coalesced stores.  The staging index is
// padded by one word per 32 so that a wave's segment reads spread over the
// LDS banks.
constexpr int kScanPer = 12;
constexpr int kScanChunk = 1024 * kScanPer;
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }

__global__ void __launch_bounds__(1024) scan_kernel(MatrixView A, int32_t* clear, int64_t clear_count) {
    __shared__ int s_val[kScanChunk + kScanChunk / 32];
    __shared__ int s_wave[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // a one-shot decode's solve control block (read only by the next kernel)
    for (int64_t i = tid; i < clear_count; i += 1024) clear[i] = 0;
    int carry = 0;
    for (int base = 0; base < A.m; base += kScanChunk) {
        const int len = min(kScanChunk, A.m - base);
        int v[kScanPer];
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            const int i = u * 1024 + tid;
            v[u] = A.deg[base + (i < len ? i : len - 1)];
        }
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            const int i = u * 1024 + tid;
            s_val[scan_pad(i)] = i < len ? v[u] : 0;
        }
        __syncthreads();
        int sum = 0;
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            v[u] = s_val[scan_pad(tid * kScanPer + u)];
            sum += v[u];
        }
        int incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        if (lane == 63) s_wave[wid] = incl;
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < 16; ++w) {
            const int t = s_wave[w];
            before += w < wid ? t : 0;
            total += t;
        }
        int run = carry + before + incl - sum;
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            s_val[scan_pad(tid * kScanPer + u)] = run;
            run += v[u];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            const int i = u * 1024 + tid;
            if (i < len) A.row_off[base + i] = s_val[scan_pad(i)];
        }
        carry += total;
        __syncthreads();  // s_val and s_wave are reused by the next chunk
    }
    if (tid == 0) A.row_off[A.m] = carry;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

hipError_t launch_zero(int32_t* p, int64_t count, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_ints, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

namespace {

uint64_t clock_khz() {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;  // 100 MHz
    return static_cast<uint64_t>(khz);
}

uint64_t barrier_limit_ticks() { return clock_khz() * 1000ull * 20ull; }  // 20 seconds

// Admission settings (process-wide): member cap (0: none) and the window in
// microseconds.  All workgroups of an idle device start within a few
// microseconds, and the last of them closes admission at once; the window
// only matters when some cannot start.
constexpr int kAdmitWindowUs = 100;
std::atomic<int> g_admit_cap{0};
std::atomic<int> g_admit_window_us{kAdmitWindowUs};

template <int D>
hipError_t prepare_d(const int32_t* col_idx, const MatrixView& A, hipStream_t s, ZeroSpan clear) {
    const int cus = device_cus();
    // the degree counts and the bad-index flag follow each other in the
    // matrix buffers: one fill clears both
    const size_t hist_bytes = static_cast<size_t>(A.m) * sizeof(int);
    const size_t stage_bytes = static_cast<size_t>(kRepackWaves) * 64 * D * sizeof(int);
    const int lds_hist = repack_lds_hist(A.m, D) ? 1 : 0;
    if (!lds_hist && (!A.partial || !A.blk)) return hipErrorInvalidValue;  // the layout has no partial counts
    if (!lds_hist) {
        // the degrees are written whole by the reduction
        hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, A.bad_input, int64_t(1));
    } else if (A.bad_input > A.deg) {
        hipLaunchKernelGGL(zero_ints, dim3(256), dim3(256), 0, s, A.deg, static_cast<int64_t>(A.bad_input - A.deg) + 1);
    } else {
        hipLaunchKernelGGL(zero_ints, dim3(256), dim3(256), 0, s, A.deg, static_cast<int64_t>(A.m));
        hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, A.bad_input, int64_t(1));
    }
    const size_t lds = (lds_hist ? hist_bytes : 0) + stage_bytes;
    const void* fn = A.rows16 ? (lds_hist ? reinterpret_cast<const void*>(&repack_kernel<D, uint16_t, true>)
                                           : reinterpret_cast<const void*>(&repack_kernel<D, uint16_t, false>))
                               : (lds_hist ? reinterpret_cast<const void*>(&repack_kernel<D, int32_t, true>)
                                           : reinterpret_cast<const void*>(&repack_kernel<D, int32_t, false>));
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const int64_t groups = A.ntiles * (kTile / 64);
    int64_t blocks = (groups + kRepackWaves - 1) / kRepackWaves;
    const int64_t cap = static_cast<int64_t>(cus > 0 ? cus : 256) * (lds_hist ? 1 : 2);
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    void* args[] = {const_cast<int32_t**>(&col_idx), const_cast<MatrixView*>(&A)};
    hipError_t e = hipLaunchKernel(fn, dim3(static_cast<unsigned>(blocks)), dim3(1024), args, lds, s);
    if (e != hipSuccess) return e;
    if (!lds_hist) {
        const void* pf = reinterpret_cast<const void*>(&deg_partial_kernel);
        const size_t plds = static_cast<size_t>(kDegRange) * sizeof(int);
        e = hipFuncSetAttribute(pf, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(plds));
        if (e != hipSuccess) return e;
        int64_t nd = A.n * D;
        void* pargs[] = {const_cast<int32_t**>(&col_idx), const_cast<MatrixView*>(&A), &nd};
        const unsigned ranges = static_cast<unsigned>((A.m + kDegRange - 1) / kDegRange);
        e = hipLaunchKernel(pf, dim3(static_cast<unsigned>(A.slices), ranges), dim3(1024), pargs, plds, s);
        if (e != hipSuccess) return e;
        const unsigned nblk = static_cast<unsigned>(deg_blocks(A.m));
        hipLaunchKernelGGL(deg_reduce_kernel, dim3(nblk), dim3(1024), 0, s, A);
        hipLaunchKernelGGL(scan_blocks_kernel, dim3(nblk), dim3(1024), 0, s, A, clear.p, clear.count);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, A, clear.p, clear.count);
    return hipGetLastError();
}

template <int D, int WM>
hipError_t solve_d(const SolveParams& p, hipStream_t s) {
    const void* fn = reinterpret_cast<const void*>(&solve_kernel<D, WM>);
    // the LDS word copy, rounded up for the 16-byte staging copies
    const size_t lds = WM == kWordsGlobal ? 0 : (static_cast<size_t>(p.m) * word_bytes(WM) + 15) / 16 * 16;
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
    // control block and per-iteration counters (adjacent in the workspace:
    // one fill clears both)
    int32_t* const ctrl_ints = reinterpret_cast<int32_t*>(p.ctrl);
    if (p.ctrl_cleared) {
        // zeroed by the preparation's scan kernel, earlier on this stream
    } else if (p.tcount >= ctrl_ints + sizeof(Ctrl) / sizeof(int32_t) && p.tcount - ctrl_ints <= 4096) {
        hipLaunchKernelGGL(zero_ints, dim3(8), dim3(256), 0, s, ctrl_ints,
                           static_cast<int64_t>(p.tcount - ctrl_ints) + 2 * (p.max_iter + 2));
    } else {
        hipLaunchKernelGGL(zero_ints, dim3(1), dim3(256), 0, s, ctrl_ints,
                           static_cast<int64_t>(sizeof(Ctrl) / sizeof(int32_t)));
        hipLaunchKernelGGL(zero_ints, dim3(8), dim3(256), 0, s, p.tcount,
                           static_cast<int64_t>(2 * (p.max_iter + 2)));
    }
    SolveParams q = p;
    Admission adm;
    adm.limit = barrier_limit_ticks();
    adm.window = clock_khz() * static_cast<uint64_t>(g_admit_window_us.load()) / 1000ull;
    const int cap = g_admit_cap.load();
    adm.cap = cap > 0 ? static_cast<unsigned>(cap) : 0xFFFFFFFFu;
    void* args[] = {&q, &adm};
    // An ordinary launch: the kernel admits the workgroups that start and
    // splits the work among them, so co-residency of the whole grid is not
    // required (a cooperative launch would add about 20 us per solve).
    return hipLaunchKernel(fn, dim3(static_cast<unsigned>(grid)), dim3(kBlock), args,
                           static_cast<unsigned>(lds), s);
}

template <int D>
hipError_t solve_dispatch_r(const SolveParams& p, hipStream_t s) {
    switch (p.wmode) {
        case kWordsLds32: return solve_d<D, kWordsLds32>(p, s);
        case kWordsLds16: return solve_d<D, kWordsLds16>(p, s);
        case kWordsLds8: return solve_d<D, kWordsLds8>(p, s);
        default: return solve_d<D, kWordsGlobal>(p, s);
    }
}

template <int D = kDMin>
hipError_t prepare_dispatch(int d, const int32_t* col_idx, const MatrixView& A, hipStream_t s,
                            ZeroSpan clear) {
    if constexpr (D > kDMax) {
        return hipErrorInvalidValue;
    } else {
        if (d == D) return prepare_d<D>(col_idx, A, s, clear);
        return prepare_dispatch<D + 1>(d, col_idx, A, s, clear);
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

hipError_t launch_prepare(const int32_t* col_idx, const MatrixView& A, int /*check*/, hipStream_t s,
                          ZeroSpan clear) {
    return prepare_dispatch(A.d, col_idx, A, s, clear);
}

ZeroSpan solve_control_span(const SolveParams& p) {
    // the one-fill case of the solve's own reset, bounded so that one
    // workgroup clears it in a few microseconds
    constexpr int64_t kMaxWords = int64_t(1) << 16;
    int32_t* const ctrl_ints = reinterpret_cast<int32_t*>(p.ctrl);
    ZeroSpan z;
    if (p.tcount >= ctrl_ints + sizeof(Ctrl) / sizeof(int32_t) && p.tcount - ctrl_ints <= 4096) {
        const int64_t count = static_cast<int64_t>(p.tcount - ctrl_ints) + 2 * (static_cast<int64_t>(p.max_iter) + 2);
        if (count <= kMaxWords) {
            z.p = ctrl_ints;
            z.count = count;
        }
    }
    return z;
}

hipError_t launch_solve(const SolveParams& p, hipStream_t s) { return solve_dispatch(p, s); }

uint64_t wait_limit_ticks() { return barrier_limit_ticks(); }

void set_solve_admission(int32_t max_members, int32_t window_us) {
    g_admit_cap.store(max_members > 0 ? max_members : 0);
    g_admit_window_us.store(window_us > 0 ? window_us : kAdmitWindowUs);
}

}  // namespace l0
