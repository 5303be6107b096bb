// Column scoring shared by the decoder's kernels: the exact score of one
// column (eq. (selection_l0)) and the bucket-word filter that lets the
// streaming vote skip the exact score for columns that cannot be selected.
// Host-callable as well, so the filter's exactness can be tested on the CPU.
#pragma once

#include <cmath>
#include <climits>
#include <cstdint>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define L0_HD __host__ __device__ __forceinline__
#else
#define L0_HD
#endif

namespace l0 {

// Scoring rules (same values as l0_rule in l0decode.h).  The shifted rules
// score one candidate per column per vote pass (Algorithm 3).
constexpr int kRuleL0dec = 0;
constexpr int kRuleMode = 1;
constexpr int kRuleShiftedL0dec = 2;
constexpr int kRuleShiftedMode = 3;

L0_HD bool rule_is_shifted(int rule) { return rule >= kRuleShiftedL0dec; }

// Rules whose score subtracts the zero entries (the l0-decrease c - z).
L0_HD bool rule_counts_zeros(int rule) { return rule == kRuleL0dec || rule == kRuleShiftedL0dec; }

// The score itself, by its definition, on the column's gathered residual
// values v[0..D): for every nonzero candidate v[t], c counts the entries u with
// |v[u] - v[t]| <= tau; the l0-decrease is c - z with z the number of zero
// entries (the frequency rule scores c).  Best score wins, ties go to the
// smallest value.  Returns true (and omega) when the best score reaches a.
template <int D>
L0_HD bool exact_score(const double (&v)[D], double tau, int rule, int a,
                                            double& omega) {
    int z = 0;
#pragma unroll
    for (int u = 0; u < D; ++u) z += !(std::fabs(v[u]) > tau);
    int top = INT_MIN;
    double w = 0.0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        if (!(std::fabs(v[t]) > tau)) continue;
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < D; ++u) cnt += !(std::fabs(v[u] - v[t]) > tau);
        const int score = (rule == kRuleMode) ? cnt : cnt - z;
        if (top == INT_MIN || score > top || (score == top && v[t] < w)) {
            top = score;
            w = v[t];
        }
    }
    omega = w;
    return top != INT_MIN && top >= a;
}

// The shifted score (Algorithm 3): the only candidate is v[t], tried when
// nonzero; c counts the entries within tau of it, the score is c - z (c for
// the frequency rule) and the column is selected when it reaches a, with
// omega = v[t].
template <int D>
L0_HD bool exact_score_shifted(const double (&v)[D], int t, double tau, int rule, int a, double& omega) {
    omega = 0.0;
    double cand = v[0];
#pragma unroll
    for (int u = 1; u < D; ++u)
        if (u == t) cand = v[u];
    if (!(std::fabs(cand) > tau)) return false;
    int z = 0, c = 0;
#pragma unroll
    for (int u = 0; u < D; ++u) {
        z += !(std::fabs(v[u]) > tau);
        c += !(std::fabs(v[u] - cand) > tau);
    }
    const int score = rule_counts_zeros(rule) ? c - z : c;
    if (score < a) return false;
    omega = cand;
    return true;
}

// ---------------------------------------------------------------------------
// row bucket words: a cheap, exact necessary condition for selection
// ---------------------------------------------------------------------------
//
// Each row i carries a 32-bit word: bit 31 marks a zero entry (|r_i| <= tau);
// bits 0..30 mark buckets of the value r_i on a grid of width W, a power of
// two with W >= 16 tau, bucket b taking bit (b mod 31).  A row also marks the
// neighbouring bucket when r_i lies within W/8 of a bucket edge.  If
// |r_u - r_t| <= tau (up to one rounding), then r_u and r_t are either in one
// bucket or straddle an edge within tau <= W/16 of both, so r_u carries the
// bucket bit of r_t.  Hence for any candidate t, the number of the column's
// words holding t's bucket bit is at least c_t, and a column can only be
// selected when some bucket bit is set in at least a + z of its words (a for
// the frequency rule).  Columns passing that test are scored exactly by
// exact_score() on FP64 values.  Any function of b alone keeps the test
// necessary; b mod 31 costs a few floating-point operations, gives adjacent
// buckets adjacent bits (cyclically), and maps unrelated values to a bit
// about uniformly.

constexpr double kEdge = 0.125;  // W/8 band at each bucket edge
constexpr uint32_t kZeroBit = 0x80000000u;
constexpr uint32_t kBucketBits = 0x7FFFFFFFu;

// b mod 31 (in 0..30) of an integer-valued double b, |b| < 2^51.  The
// quotient estimate is within one of floor(b / 31), the fused remainder is
// exact (a small integer), and one correction either way makes it the
// remainder.
L0_HD uint32_t bucket_index(double b) {
    const double t = std::floor(b * (1.0 / 31.0));
    double r = std::fma(-31.0, t, b);
    if (r < 0.0) r += 31.0;
    if (r >= 31.0) r -= 31.0;
    return static_cast<uint32_t>(r);
}

L0_HD uint32_t row_word(double r, double tau, double inv_w) {
    uint32_t w = (std::fabs(r) > tau) ? 0u : kZeroBit;
    const double q = r * inv_w;  // exact: inv_w is a power of two
    if (!(std::fabs(q) < 0x1p51)) return w | kBucketBits;  // huge or non-finite: every bucket
    const double b = std::floor(q);
    const double f = q - b;      // exact, in [0, 1)
    const uint32_t k = bucket_index(b);
    const uint32_t bit = 1u << k;
    w |= bit;
    if (f < kEdge) w |= k == 0u ? (1u << 30) : (bit >> 1);        // bucket b - 1
    if (f > 1.0 - kEdge) w |= k == 30u ? 1u : (bit << 1);         // bucket b + 1
    return w;
}

// Bucket width: the smallest power of two >= 16 tau (tau > 0), or a grid
// fine relative to max |y| when tau = 0 (exact equality needs no width).
L0_HD double bucket_width(double tau, double ymax) {
    double base = tau > 0.0 ? 16.0 * tau : ymax * 0x1p-44;
    if (!(base > 0x1p-1000)) base = 0x1p-1000;
    if (!(base < 0x1p1000)) base = 0x1p1000;
    int e = 0;
    (void)std::frexp(base, &e);  // base = f * 2^e, f in [0.5, 1)
    return std::ldexp(1.0, e);
}

// 16-bit words for LDS copies of up to twice as many rows: bucket bit k of
// a 32-bit word goes to bit k mod 15, the zero flag to bit 15.  Folding maps
// a word holding t's bucket bit to one holding t's folded bit, so counts per
// folded bit are never below the counts per original bit: the filter on
// unfolded words stays a necessary condition (it only passes more columns).
L0_HD uint16_t fold_word(uint32_t w) {
    const uint32_t b = (w & 0x7FFFu) | ((w >> 15) & 0x7FFFu) | ((w >> 30) & 1u);
    return static_cast<uint16_t>(b | ((w >> 16) & 0x8000u));
}

// A folded word back in the 32-bit layout (zero flag in bit 31).
L0_HD uint32_t unfold_word(uint16_t h) {
    return (static_cast<uint32_t>(h) & 0x7FFFu) | ((static_cast<uint32_t>(h) & 0x8000u) << 16);
}

// 8-bit words for LDS copies of up to four times as many rows: bucket bit k
// goes to bit k mod 7, the zero flag to bit 7.  The same argument as for the
// 16-bit fold keeps the filter a necessary condition.
L0_HD uint8_t fold_word8(uint32_t w) {
    const uint32_t v = w & kBucketBits;
    uint32_t b = 0u;
#pragma unroll
    for (int s = 0; s < 31; s += 7) b |= (v >> s) & 0x7Fu;
    return static_cast<uint8_t>(b | ((w >> 24) & 0x80u));
}

// An 8-bit folded word back in the 32-bit layout (zero flag in bit 31).
L0_HD uint32_t unfold_word8(uint8_t h) {
    return (static_cast<uint32_t>(h) & 0x7Fu) | ((static_cast<uint32_t>(h) & 0x80u) << 24);
}

// Bit-sliced population count of D words: c[k] holds bit k of the per-bit-
// position count.  Full adders (xor / majority) for the common degrees, a
// ripple-carry accumulation otherwise.
template <int D>
struct Levels {
    static constexpr int L = D >= 16 ? 5 : D >= 8 ? 4 : D >= 4 ? 3 : D >= 2 ? 2 : 1;
};

L0_HD void full_add(uint32_t a, uint32_t b, uint32_t c, uint32_t& s, uint32_t& cy) {
#if defined(__HIP_DEVICE_COMPILE__)
    // one three-input bitwise instruction each (truth tables: parity 0x96,
    // majority 0xE8)
    s = __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
    cy = __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
#else
    const uint32_t x = a ^ b;
    s = x ^ c;
    cy = (x & c) | (~x & a);
#endif
}

template <int D>
L0_HD void bit_count(const uint32_t (&w)[D], uint32_t (&c)[Levels<D>::L]) {
    constexpr int L = Levels<D>::L;
    if constexpr (D == 7) {
        uint32_t s1, c1, s2, c2, c3, c4;
        full_add(w[0], w[1], w[2], s1, c1);
        full_add(w[3], w[4], w[5], s2, c2);
        full_add(s1, s2, w[6], c[0], c3);
        full_add(c1, c2, c3, c[1], c4);
        c[2] = c4;
    } else if constexpr (D == 5) {
        uint32_t s1, c1, c2;
        full_add(w[0], w[1], w[2], s1, c1);
        full_add(s1, w[3], w[4], c[0], c2);
        c[1] = c1 ^ c2;
        c[2] = c1 & c2;
    } else if constexpr (D == 9) {
        uint32_t s1, c1, s2, c2, s3, c3, c4, t1, c5, c6;
        full_add(w[0], w[1], w[2], s1, c1);
        full_add(w[3], w[4], w[5], s2, c2);
        full_add(w[6], w[7], w[8], s3, c3);
        full_add(s1, s2, s3, c[0], c4);
        full_add(c1, c2, c3, t1, c5);
        c[1] = t1 ^ c4;
        c6 = t1 & c4;
        c[2] = c5 ^ c6;
        c[3] = c5 & c6;
    } else {
#pragma unroll
        for (int k = 0; k < L; ++k) c[k] = 0u;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            uint32_t carry = w[i];
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const uint32_t t = c[k] & carry;
                c[k] ^= carry;
                carry = t;
            }
        }
    }
}

// True when some bucket bit is set in at least a + z words (a words for the
// frequency rule), z being the count of zero entries (bit 31).
template <int D>
L0_HD bool bucket_filter(const uint32_t (&w)[D], int a, int rule) {
    constexpr int L = Levels<D>::L;
    uint32_t c[L];
    bit_count<D>(w, c);
    int z = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) z |= static_cast<int>(c[k] >> 31) << k;
    const int need = a + (rule_counts_zeros(rule) ? z : 0);
    // need > D can never be met; tested without a branch (the carry chain
    // below then sees a wrapped constant, and its result is discarded)
    const bool reachable = need <= D;
    // count >= need exactly when count + (2^L - need) carries out of L bits
    // (for 1 <= need <= D < 2^L the constant lies in [1, 2^L)): the carry
    // chain of that addition on the bit-sliced counts, one majority per level
    const int K = (1 << L) - need;
    // bit k of K as an all-ones or all-zero mask
    auto kmask = [K](int k) { return static_cast<uint32_t>(-((K >> k) & 1)); };
    uint32_t carry = c[0] & kmask(0);
#pragma unroll
    for (int k = 1; k < L; ++k) {
#if defined(__HIP_DEVICE_COMPILE__)
        carry = __builtin_amdgcn_bitop3_b32(c[k], carry, kmask(k), 0xE8);  // majority
#else
        const uint32_t kb = kmask(k);
        carry = (c[k] & carry) | (kb & (c[k] | carry));
#endif
    }
    return reachable & ((carry & kBucketBits) != 0u);
}


}  // namespace l0
