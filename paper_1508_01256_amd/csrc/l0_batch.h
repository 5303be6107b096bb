// Internal declarations of the batched decoder (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "l0_internal.h"

namespace l0 {

// Byte offsets, within one instance's scratch region, of its working arrays
// (sized by that instance alone).
struct InstLayout {
    size_t r, rword, member, slot_cnt, slot_sorted, aff_flag, aff_list, row_off, slots, overflow, soa;
    size_t total;
};

__host__ __device__ inline size_t align256_hd(size_t b) { return (b + 255) & ~size_t(255); }

// The instance's repacked index store, which its votes stream: chunks of 64
// 32-bit words per neighbour plane.  16-bit rows (m <= 65536): a chunk holds
// 128 columns, word w of plane t the t-th rows of columns 2w (low half) and
// 2w + 1 (high half); 32-bit rows: 64 columns, word w the row of column w.
// Chunk c's plane t starts at 32-bit word (c*d + t)*64.
__host__ __device__ inline bool batch_rows16(int32_t m) { return m <= 65536; }
__host__ __device__ inline int64_t batch_chunk_cols(int32_t m) { return batch_rows16(m) ? 128 : 64; }
__host__ __device__ inline int64_t batch_chunks(int64_t n, int32_t m) {
    return (n + batch_chunk_cols(m) - 1) / batch_chunk_cols(m);
}

__host__ __device__ inline InstLayout inst_layout(int64_t n, int32_t m, int32_t d) {
    const int64_t nd = n * d;
    InstLayout L{};
    size_t o = 0;
    L.r = o;
    o += align256_hd(static_cast<size_t>(m) * 8);
    L.rword = o;
    o += align256_hd(static_cast<size_t>(m) * 4);
    L.member = o;
    o += align256_hd(static_cast<size_t>((n + 31) / 32) * 4);
    L.slot_cnt = o;
    o += align256_hd(static_cast<size_t>(m) * 4);
    L.slot_sorted = o;
    o += align256_hd(static_cast<size_t>(m) * 4);
    L.aff_flag = o;
    o += align256_hd(static_cast<size_t>(m) * 4);
    L.aff_list = o;  // two lists (iteration parity)
    o += align256_hd(static_cast<size_t>(m) * 8);
    L.row_off = o;
    o += align256_hd((static_cast<size_t>(m) + 1) * 4);
    L.slots = o;
    o += align256_hd(static_cast<size_t>(nd) * 4);
    L.overflow = o;
    o += align256_hd(static_cast<size_t>(n) * 4);
    L.soa = o;
    o += static_cast<size_t>(batch_chunks(n, m)) * d * 256;
    L.total = o;
    return L;
}

// Counters of one iteration shared by an instance's team.  Iteration l uses
// ring[l % 3]; the leader clears ring[(l + 1) % 3] during iteration l.
struct IterCounters {
    int tcount;  // |T_l|
    int affc;    // touched rows
    int spill;   // columns in the shared overflow list
    int delta;   // change of ||r||_0
};

// Control block of one instance (zeroed before the launch).
struct alignas(256) TeamCtl {
    int bar;      // team barrier arrivals (monotonic)
    int abort;    // a barrier wait timed out
    int bad;      // input errors (kErr* bits)
    int nnz;      // ||y||_0
    unsigned long long ymax_bits;  // max |y_i| (bits of a non-negative double)
    int support;  // |support|
    int pad0;
    IterCounters ring[3];
};

// Work items: instance index in the low 23 bits, team member in the high 8.
constexpr int kItemInstBits = 23;
constexpr int kMaxTeam = 256;

struct BatchParams {
    const l0_problem* probs;  // device copy of the instance table
    const int32_t* items;     // this launch's work items, in claim order
    const int32_t* team;      // team size per instance
    const int64_t* inst_off;  // scratch offset per instance
    int32_t count;            // work items in this launch
    int32_t rule;
    int32_t tol_mode;
    int32_t words_cap;        // bucket words kept in LDS when m <= words_cap
    int32_t stage_d;          // largest degree in the launch (LDS staging size)
    l0_result* results;
    char* scratch;            // instance scratch regions
    TeamCtl* ctl;             // one per instance
    unsigned* next;           // work counter (zeroed before the launch)
    int64_t* timing;          // optional per-instance timing records (8 int64 each)
    uint64_t wait_limit;      // bound of one team-barrier wait, in device clock ticks
};

// LDS bytes of the batched kernel for a block size, word capacity and degree.
size_t batch_lds_bytes(int block_threads, int words_cap, int d);

// Degree ranges with a kernel of their own (inclusive bounds).
constexpr int kBatchRangeCount = 4;
constexpr int kBatchRanges[kBatchRangeCount][2] = {{2, 4}, {5, 9}, {10, 14}, {15, 20}};

inline int batch_range_of(int d) {
    for (int r = 0; r < kBatchRangeCount; ++r)
        if (d >= kBatchRanges[r][0] && d <= kBatchRanges[r][1]) return r;
    return -1;
}

// The kernel for a block size (256 or 512 threads) and degree range, or
// nullptr.
const void* batch_kernel_fn(int block_threads, int range);

// l0_decode_batched planned within 1/share of the device's resident
// workgroups (grid and teams), for callers that run up to `share` batches on
// the device at once: they can then all be resident together, so no team
// waits for members that cannot be scheduled.
l0_status decode_batched_share(const l0_problem* probs, int32_t count, const l0_batch_opts* opts,
                               l0_result* results, void* workspace, size_t ws_bytes, hipStream_t stream,
                               int share);

}  // namespace l0
