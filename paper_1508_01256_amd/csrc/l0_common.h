// Device helpers shared by the single-instance and the batched decoders:
// applying one selected update (Algorithm 2's x_hat_j += omega) and
// recomputing one residual entry (r <- y - A x_hat, row by row).  The state
// record's pointers may be generic or typed global-memory pointers; the
// atomics are the relaxed, device-scope operations of HIP's atomicAdd,
// atomicOr and atomicExch, written so that they accept either.
#pragma once

#include <hip/hip_runtime.h>
#include <climits>
#include <stdint.h>

namespace l0 {

// Number of lanes of this wave with `pred`, in every lane (wave ballot).
__device__ __forceinline__ int wave_count(bool pred) {
    return __popcll(__ballot(pred));
}

template <class Ptr, class V>
__device__ __forceinline__ V fetch_add(Ptr p, V v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Column j's term in a residual row: x_hat_j, or the rounded product
// w_j * x_hat_j on a column-scaled A (S provides x and w).
template <class S>
__device__ __forceinline__ double column_term(const S& p, int64_t j) {
    const double xj = p.x[j];
    return p.w ? p.w[j] * xj : xj;
}

// The update of column j that cancels residual value v: v, or v / w_j on a
// column-scaled A (w_j > 0).
template <class S>
__device__ __forceinline__ double column_update(const S& p, int64_t j, double v) {
    return p.w ? v / p.w[j] : v;
}

// Apply x_hat_j += w for a selected column j with rows rows[0..D): count it in
// *tcount, enter j into the support (bitmap; on first entry append j to each
// row's support list and count it in *support), and record every row it
// touches once in the touched-row list (count in *affc).  S provides x,
// member, slot_cnt, slots, row_off, aff_flag, aff_list.  Two rounds of
// memory operations, each issued together: the support bit, the touched-row
// flags, the rows' list offsets and x_hat_j; then, knowing which of these
// are first, the list slots and the touched-row positions.
template <int D, class S, class C>
__device__ void apply_update(const S& p, C tcount, C support, C affc, int64_t j, double w,
                             const int (&rows)[D]) {
    const double x0 = p.x[j];
    fetch_add(tcount, 1);
    const uint32_t bit = 1u << (j & 31);
    const uint32_t old = __hip_atomic_fetch_or(&p.member[j >> 5], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int first[D], off[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        first[t] = __hip_atomic_exchange(&p.aff_flag[rows[t]], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        off[t] = p.row_off[rows[t]];
    }
    const bool fresh = (old & bit) == 0;
    int nfirst = 0;
#pragma unroll
    for (int t = 0; t < D; ++t) nfirst += first[t] == 0;
    int q[D];
    if (fresh) {
        fetch_add(support, 1);
#pragma unroll
        for (int t = 0; t < D; ++t) q[t] = fetch_add(&p.slot_cnt[rows[t]], 1);
    }
    int qa = 0;
    if (nfirst) qa = fetch_add(affc, nfirst);
    if (fresh) {
#pragma unroll
        for (int t = 0; t < D; ++t) p.slots[off[t] + q[t]] = static_cast<int>(j);
    }
    if (nfirst) {
#pragma unroll
        for (int t = 0; t < D; ++t)
            if (first[t] == 0) p.aff_list[qa++] = rows[t];
    }
    p.x[j] = x0 + w;
}

// r_i = y_i - (sum over the support columns of row i, ascending, of their
// column terms).  The row's list holds its support columns; entries appended
// since the last visit are merged into the sorted prefix first.
template <class S>
__device__ double row_residual(const S& p, int i) {
    const auto list = p.slots + p.row_off[i];
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
    for (int q = 0; q < cnt; ++q) s += column_term(p, list[q]);
    return p.y[i] - s;
}

// Support lists of at most this many entries are sorted in registers.
constexpr int kShortList = 16;

// Ascending bitonic sorting network over N (a power of two) register values.
template <int N>
__device__ __forceinline__ void sort_network(int (&v)[N]) {
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const int a = v[i], b = v[l];
                    const bool up = (i & k) == 0;
                    v[i] = up ? min(a, b) : max(a, b);
                    v[l] = up ? max(a, b) : min(a, b);
                }
            }
        }
    }
}

// row_residual for a row whose support list holds cnt <= N entries (N a
// power of two): the list is sorted in registers (and written back) when it
// has unsorted entries, the column terms are gathered for all entries at
// once, and the sum still runs in ascending j from +0.0.
template <int N, class S>
__device__ double row_residual_short(const S& p, int i, int cnt) {
    const auto list = p.slots + p.row_off[i];
    int v[N];
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = q < cnt ? list[q] : INT_MAX;
    if (p.slot_sorted[i] != cnt) {
        sort_network<N>(v);
#pragma unroll
        for (int q = 0; q < N; ++q)
            if (q < cnt) list[q] = v[q];
        p.slot_sorted[i] = cnt;
    }
    double xv[N];
#pragma unroll
    for (int q = 0; q < N; ++q) xv[q] = q < cnt ? column_term(p, v[q]) : 0.0;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (q < cnt) s += xv[q];
    return p.y[i] - s;
}

// row_residual by list length: the plain merge for one or two entries
// (nothing to gain), register networks of 4, 8 or 16 entries, the plain
// merge again above kShortList.
template <class S>
__device__ double row_residual_any(const S& p, int i, int cnt) {
    if (cnt <= 2 || cnt > kShortList) return row_residual(p, i);
    if (cnt <= 4) return row_residual_short<4>(p, i, cnt);
    if (cnt <= 8) return row_residual_short<8>(p, i, cnt);
    return row_residual_short<16>(p, i, cnt);
}

}  // namespace l0
