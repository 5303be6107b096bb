// Internal declarations of the batched decoder (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "l0_internal.h"

namespace l0 {

// Byte offsets of one workgroup's scratch (sized for the batch's largest
// instance; a workgroup solves one instance at a time).
struct BatchLayout {
    size_t r, rword, member, slot_cnt, slot_sorted, aff_flag, aff_list, long_rows, row_off, slots, overflow;
    size_t stride;
};

struct BatchParams {
    const l0_problem* probs;  // device copy of the instance table
    const int32_t* order;     // this launch's instances, largest first
    int32_t count;
    int32_t rule;
    int32_t tol_mode;
    int32_t words_cap;        // bucket words kept in LDS when m <= words_cap
    int32_t stage_d;          // largest degree in the launch (LDS staging size)
    l0_result* results;
    char* scratch;            // one BatchLayout per resident workgroup
    BatchLayout lay;
    unsigned* next;           // work counter (zeroed before the launch)
    int64_t* timing;          // optional per-instance timing records (8 int64 each)
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

}  // namespace l0
