// Internal declarations shared by the host API and the device code of the
// Parallel-l0 decoder.  Not part of the public C-ABI (include/l0decode.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "l0decode.h"

namespace l0 {

constexpr int kDMin = 2;
constexpr int kDMax = 20;
constexpr int kTile = 256;          // columns per tile of the repacked index store
constexpr int kBlock = 1024;        // threads per workgroup of the solve kernel
constexpr int kWaves = kBlock / 64; // wavefronts per workgroup
// LDS bytes for the row bucket words of the vote (gfx950 has 160 KiB per CU;
// the rest holds the per-workgroup queue and reduction scratch).
constexpr size_t kLdsWordBytes = 144 * 1024;

// How a solve keeps the bucket words its vote gathers:
//   kWordsLds32   m <= 36864:  32-bit words in LDS
//   kWordsLds16   m <= 65536:  16-bit folded words in LDS
//   kWordsLds8    m <= 147456: 8-bit folded words in LDS
//   kWordsGlobal  larger m:    32-bit words gathered from global memory
// The global copy of the words (maintained by the residual phase) has the
// same width as the LDS copy.
constexpr int kWordsGlobal = 0;
constexpr int kWordsLds32 = 1;
constexpr int kWordsLds16 = 2;
constexpr int kWordsLds8 = 3;
constexpr int word_bytes(int wm) { return wm == kWordsLds16 ? 2 : (wm == kWordsLds8 ? 1 : 4); }
inline int word_mode(int32_t m) {
    const size_t mm = static_cast<size_t>(m);
    if (mm * 4 <= kLdsWordBytes) return kWordsLds32;
    if (mm <= 65536 && mm * 2 <= kLdsWordBytes) return kWordsLds16;
    if (mm <= kLdsWordBytes) return kWordsLds8;
    return kWordsGlobal;
}
// Row indices are stored as 16 bits when every row fits.
inline bool rows16(int32_t m) { return m <= 65536; }

// Degree counting of the matrix preparation.  The repack kernel (waves of
// kRepackWaves per workgroup, each staging 64 columns) counts row degrees in
// an LDS histogram when m counts fit beside its staging area.  Otherwise
// the index array is cut into deg_slices(...) slices and the rows into ranges
// of kDegRange; one workgroup per slice and range counts in LDS and writes
// dense partial counts, which a reduction sums per row (with totals per 1024
// rows, from which the prefix sum is formed by all workgroups at once): no
// global atomics (one per index was 0.3 ms at n = 2^20, m = 104858).
constexpr int kRepackWaves = 16;
constexpr int kDegRange = 36864;  // rows per LDS pass of the partial counts (144 KiB)
inline bool repack_lds_hist(int32_t m, int32_t d) {
    return static_cast<size_t>(m) * 4 + static_cast<size_t>(kRepackWaves) * 64 * d * 4 <= kLdsWordBytes;
}
inline int64_t deg_blocks(int32_t m) { return (static_cast<int64_t>(m) + 1023) / 1024; }
inline int deg_slices(int64_t n, int32_t d) {
    const int64_t s = n * d / 8192;  // at least 8192 indices per slice
    return static_cast<int>(s < 1 ? 1 : (s > 64 ? 64 : s));
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Device-resident prepared matrix (layout of the repacked column-index store):
//   soa[(tile*d + t)*kTile + c] = row of column tile*kTile + c, t-th neighbour
// as uint16 when rows16(m), else int32 (columns past n hold row 0 and are
// never scored); row_off[i] .. row_off[i+1] is row i's capacity region in the
// per-row support lists (its degree in A).
struct MatrixView {
    int64_t n;
    int32_t m;
    int32_t d;
    int64_t ntiles;
    int32_t rows16;     // rows16(m): 16-bit row indices
    void* soa;
    int32_t* row_off;   // int32[m+1]
    int32_t* deg;       // int32[m] scratch for the degree histogram
    int32_t* bad_input; // int32[1]: kErrBadIndex / kErrRepeatedRow bits found while repacking
    int32_t* partial;   // int32[slices*m] partial degree counts, or nullptr (LDS histogram)
    int32_t* blk;       // int32[deg_blocks(m)] degree totals per 1024 rows (with partial)
    int32_t slices;     // slices of the index array counted apart (0: LDS histogram)
};

struct MatrixBuffers {
    size_t soa, row_off, deg, flag, partial, blk, total;
};
MatrixBuffers matrix_layout(int64_t n, int32_t m, int32_t d);

// Input errors found on the device, as bits of a flag word (several may be
// found at once); the outcome reported is the first of: row index out of
// range, a row listed twice in one column, non-finite y, column weight not
// positive and finite.
constexpr int kErrNonfiniteY = 1;
constexpr int kErrBadIndex = 2;
constexpr int kErrBadWeight = 4;
constexpr int kErrRepeatedRow = 8;
__host__ __device__ inline int error_outcome(int flags) {
    return (flags & kErrBadIndex) ? L0_DEV_BAD_INDEX
         : (flags & kErrRepeatedRow) ? L0_DEV_REPEATED_ROW
         : (flags & kErrNonfiniteY) ? L0_DEV_NONFINITE_Y : L0_DEV_BAD_WEIGHT;
}

// True when two of the d row indices r[0..D) are equal (a column of a
// binary A lists each of its rows once, Definition 2.2).
template <int D>
__host__ __device__ inline bool has_repeat(const int (&r)[D]) {
    bool rep = false;
#pragma unroll
    for (int t = 1; t < D; ++t)
#pragma unroll
        for (int u = 0; u < t; ++u) rep |= r[u] == r[t];
    return rep;
}

// A usable column weight: positive and finite.
__host__ __device__ inline bool weight_ok(double w) { return w > 0.0 && w <= 1.7976931348623157e308; }

// Control block at the start of the solve workspace (zeroed before each solve).
constexpr int kMaxXcc = 16;     // XCDs (accelerator complex dies) a device may have
constexpr int kXccStride = 32;  // per-XCD counters sit 128 bytes apart
struct Ctrl {
    unsigned int bar;        // grid barrier: arrivals of each XCD's last arriver (monotonic)
    int abort;               // set when a barrier timed out
    int err;                 // device-detected input errors (kErr* bits), 0 if none
    int nnz;                 // running ||r||_0
    unsigned long long maxabs_bits; // bits of max_i |y_i| (non-negative doubles order as integers)
    int support;             // columns ever updated
    int pad0;
    long long updates;       // sum of |T| over iterations
    unsigned int start;      // start-up arrivals (every member once)
    unsigned int admit;      // admission: registrations, kClosed once closed
    unsigned int members;    // admitted workgroups, 0 until decided
    int pad[21];
    unsigned int xcount[kMaxXcc];                 // workgroups resident on each XCD
    unsigned int xarrive[kMaxXcc * kXccStride];   // per-XCD barrier arrivals (monotonic)
};

struct SolveBuffers {
    size_t ctrl, counters, r, rword, slot_cnt, slot_sorted, aff_flag, aff_list, member, slots, total;
};
SolveBuffers solve_layout(int64_t n, int32_t m, int32_t d, int32_t max_iter);

struct SolveParams {
    // problem
    int64_t n;
    int32_t m;
    int32_t d;
    int64_t ntiles;
    int32_t wmode;      // word_mode(m) (fixes the row width too)
    const void* soa;
    const int32_t* row_off;
    const int32_t* bad_input;
    const double* y;
    double tol;
    int32_t a;          // ceil(alpha)
    int32_t max_iter;
    int32_t rule;
    int32_t tol_mode;
    const double* x_init;
    const double* w;     // column weights of a column-scaled A, or nullptr
    // outputs
    double* x;
    int32_t* trace;
    int64_t* tsize;
    int64_t* timeline;   // optional: wall clock at start and after each grid barrier
    l0_result* res;
    int32_t* iters_out;  // optional (plain l0_decode)
    // workspace
    Ctrl* ctrl;
    int32_t* tcount;     // int32[max_iter+2]
    int32_t* affc;       // int32[max_iter+2]
    double* r;
    void* rword;         // m bucket words of the residual entries, word_bytes(wmode) each
    int32_t* slot_cnt;
    int32_t* slot_sorted;
    int32_t* aff_flag;
    int32_t* aff_list;   // int32[2m]: touched rows of even / odd iterations
    uint32_t* member;
    int32_t* slots;
    // the control block and counters are already zero (a one-shot decode
    // has the preparation clear them), so the solve launches no fill
    int32_t ctrl_cleared;
};

// A run of int32 words to zero, or none (p == nullptr).
struct ZeroSpan {
    int32_t* p = nullptr;
    int64_t count = 0;
};

// The solve's control block and per-iteration counters as one run of words,
// when they are adjacent and the run is short enough for the scan kernel to
// clear (one-shot decodes); none otherwise.
ZeroSpan solve_control_span(const SolveParams& p);

// Enqueue the matrix preparation (repack, range check, degree histogram,
// scan); the scan kernel also zeroes `clear`.
hipError_t launch_prepare(const int32_t* col_idx, const MatrixView& A, int check, hipStream_t s,
                          ZeroSpan clear = ZeroSpan());

// Enqueue one solve (control reset + the persistent kernel).
hipError_t launch_solve(const SolveParams& p, hipStream_t s);

// Admission of the solve kernel's workgroups: at most max_members members
// (0: no cap), admission closed by the first member after window_us
// microseconds (<= 0: the default).
void set_solve_admission(int32_t max_members, int32_t window_us);

// Enqueue a fill of count int32 zeros (a kernel, so it may sit in graphs).
hipError_t launch_zero(int32_t* p, int64_t count, hipStream_t s);

// Compute units of the current device (0 if unknown).
int device_cus();

// Bound of one device-side wait (20 s) in ticks of the device's constant clock.
uint64_t wait_limit_ticks();

// A device-accessible buffer of at least `bytes` at p (the C-ABI's check).
bool device_buffer_ok(const void* p, size_t bytes);

}  // namespace l0
