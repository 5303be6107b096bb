// CPU property check of the decoder's column scoring (csrc/l0_filter.h):
//  1. bit_count<D> equals a naive per-bit population count;
//  2. bucket_filter<D> equals its definition on random words;
//  3. exact_score<D> equals the l0-decrease eq. (selection_l0) formed entry
//     by entry, best score first and smallest value on ties;
//  4. the filter (on 32-bit words, and on words folded to 16 and to 8 bits)
//     never rejects a column exact_score selects, on adversarial
//     columns (clusters within tau, zeros, tiny values, values straddling
//     bucket edges) for several tau, both rules and every threshold;
//  5. bucket_index is the integer remainder mod 31 over the whole bucket
//     range (|b| < 2^51): near multiples of 31, near the range's ends, near
//     powers of two, and at random.
// Exit status 0 and "OK" on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "l0_filter.h"

using namespace l0;

static std::mt19937_64 rng(12345);

template <int D>
static int check_counts(int trials) {
    constexpr int L = Levels<D>::L;
    for (int it = 0; it < trials; ++it) {
        uint32_t w[D];
        for (int t = 0; t < D; ++t) {
            // sparse-ish words like bucket words, sometimes dense
            uint32_t x = (uint32_t)rng();
            if (rng() % 4) x &= (uint32_t)rng() & (uint32_t)rng();
            w[t] = x;
        }
        uint32_t c[L];
        bit_count<D>(w, c);
        for (int b = 0; b < 32; ++b) {
            int naive = 0, got = 0;
            for (int t = 0; t < D; ++t) naive += (w[t] >> b) & 1u;
            for (int k = 0; k < L; ++k) got |= (int)((c[k] >> b) & 1u) << k;
            if (naive != got) { std::printf("bit_count D=%d mismatch\n", D); return 1; }
        }
        for (int rule = 0; rule < 2; ++rule)
            for (int a = 2; a <= D; ++a) {
                int z = 0;
                for (int t = 0; t < D; ++t) z += (w[t] >> 31) & 1u;
                const int need = a + (rule == kRuleL0dec ? z : 0);
                bool naive = false;
                for (int b = 0; b < 31; ++b) {
                    int cnt = 0;
                    for (int t = 0; t < D; ++t) cnt += (w[t] >> b) & 1u;
                    naive |= cnt >= need;
                }
                if (naive != bucket_filter<D>(w, a, rule)) {
                    std::printf("bucket_filter D=%d a=%d rule=%d mismatch\n", D, a, rule);
                    return 1;
                }
            }
    }
    return 0;
}

static double uniform(double lo, double hi) {
    return lo + (hi - lo) * (double)(rng() >> 11) * (1.0 / 9007199254740992.0);
}

template <int D>
static int check_exactness(int trials) {
    const double ymax = 3.0;
    const double taus[] = {0.0, 1e-10 * ymax, 1e-6 * ymax, 1e-3 * ymax, 0x1p-40, 0.37};
    long selected = 0, passed = 0, folded_passed = 0, folded8_passed = 0;
    for (double tau : taus) {
        const double width = bucket_width(tau, ymax);
        const double inv_w = 1.0 / width;
        for (int it = 0; it < trials; ++it) {
            double v[D];
            // a cluster centre, possibly on a bucket edge, possibly tiny
            double centre;
            switch (rng() % 5) {
                case 0: centre = uniform(-ymax, ymax); break;
                case 1: centre = std::floor(uniform(-ymax, ymax) * inv_w) * width; break;
                case 2: centre = (std::floor(uniform(-ymax, ymax) * inv_w) + 0.5) * width; break;
                case 3: centre = uniform(-2.5, 2.5) * (tau > 0 ? tau : 1e-300); break;
                default: centre = (double)(int)(rng() % 5) - 2.0; break;
            }
            const int csize = (int)(rng() % (D + 1));
            for (int t = 0; t < D; ++t) {
                const int kind = (int)(rng() % 6);
                if (t < csize || kind == 0) v[t] = centre + uniform(-1.0, 1.0) * tau;
                else if (kind == 1) v[t] = 0.0;
                else if (kind == 2) v[t] = uniform(-1.0, 1.0) * tau;
                else if (kind == 3) v[t] = centre + uniform(-2.2, 2.2) * tau;
                else v[t] = uniform(-ymax, ymax);
            }
            for (int t = D - 1; t > 0; --t) { int u = (int)(rng() % (t + 1)); double x = v[t]; v[t] = v[u]; v[u] = x; }
            uint32_t w[D];
            for (int t = 0; t < D; ++t) w[t] = row_word(v[t], tau, inv_w);
            for (int rule = 0; rule < 2; ++rule)
                for (int a = 2; a <= D; ++a) {
                    // definition: decrease of ||r||_0 over the column's rows
                    // (rules 0, 1; their shifted forms 2, 3 below)
                    int best = INT_MIN;
                    double wbest = 0.0;
                    for (int t = 0; t < D; ++t) {
                        if (!(std::fabs(v[t]) > tau)) continue;
                        int before = 0, after = 0, freq = 0;
                        for (int u = 0; u < D; ++u) {
                            before += std::fabs(v[u]) > tau;
                            const double dlt = v[u] - v[t];
                            after += std::fabs(dlt) > tau;
                            freq += !(std::fabs(dlt) > tau);
                        }
                        const int sc = rule == kRuleMode ? freq : before - after;
                        if (best == INT_MIN || sc > best || (sc == best && v[t] < wbest)) { best = sc; wbest = v[t]; }
                    }
                    const bool sel_def = best != INT_MIN && best >= a;
                    double omega = 0.0;
                    const bool sel = exact_score<D>(v, tau, rule, a, omega);
                    if (sel != sel_def || (sel && omega != wbest)) {
                        std::printf("exact_score D=%d mismatch\n", D);
                        return 1;
                    }
                    const bool pass = bucket_filter<D>(w, a, rule);
                    selected += sel;
                    passed += pass;
                    if (sel && !pass) {
                        std::printf("FILTER REJECTED A SELECTED COLUMN D=%d tau=%g a=%d rule=%d\n", D, tau, a, rule);
                        for (int t = 0; t < D; ++t) std::printf("  v=%.17g w=%08x\n", v[t], w[t]);
                        return 1;
                    }
                    // folded 16-bit words: the filter passes at least what the
                    // 32-bit filter passes (so every selected column)
                    uint32_t wf[D];
                    for (int t = 0; t < D; ++t) {
                        wf[t] = unfold_word(fold_word(w[t]));
                        if ((wf[t] >> 31) != (w[t] >> 31)) { std::printf("fold lost the zero flag\n"); return 1; }
                    }
                    const bool fpass = bucket_filter<D>(wf, a, rule);
                    folded_passed += fpass;
                    if (pass && !fpass) {
                        std::printf("FOLDED FILTER REJECTED A PASSING COLUMN D=%d tau=%g a=%d rule=%d\n", D, tau, a,
                                    rule);
                        return 1;
                    }
                    // 8-bit folds (of the 32-bit words): a word holding
                    // bucket bit k holds 8-bit bit (k mod 7) too, so they
                    // pass what the 32-bit words pass
                    uint32_t w8[D];
                    for (int t = 0; t < D; ++t) {
                        w8[t] = unfold_word8(fold_word8(w[t]));
                        if ((w8[t] >> 31) != (w[t] >> 31)) { std::printf("fold8 lost the zero flag\n"); return 1; }
                        if ((w8[t] & 0x7FFFFF80u) != 0u) { std::printf("fold8 left high bucket bits\n"); return 1; }
                    }
                    const bool f8pass = bucket_filter<D>(w8, a, rule);
                    folded8_passed += f8pass;
                    if (pass && !f8pass) {
                        std::printf("8-BIT FOLDED FILTER REJECTED A PASSING COLUMN D=%d tau=%g a=%d rule=%d\n", D,
                                    tau, a, rule);
                        return 1;
                    }
                    // shifted rule (Algorithm 3): candidate v[t] only, by its
                    // definition; the filter (with the shifted rule's zero
                    // term) must pass every column it selects
                    const int srule = rule + 2;
                    for (int t = 0; t < D; ++t) {
                        bool sdef = false;
                        if (std::fabs(v[t]) > tau) {
                            int before = 0, after = 0, freq = 0;
                            for (int u = 0; u < D; ++u) {
                                before += std::fabs(v[u]) > tau;
                                const double dlt = v[u] - v[t];
                                after += std::fabs(dlt) > tau;
                                freq += !(std::fabs(dlt) > tau);
                            }
                            sdef = (rule == kRuleMode ? freq : before - after) >= a;
                        }
                        double som = 0.0;
                        const bool ssel = exact_score_shifted<D>(v, t, tau, srule, a, som);
                        if (ssel != sdef || (ssel && som != v[t])) {
                            std::printf("exact_score_shifted D=%d t=%d mismatch\n", D, t);
                            return 1;
                        }
                        if (ssel && (!bucket_filter<D>(w, a, srule) || !bucket_filter<D>(wf, a, srule) ||
                                     !bucket_filter<D>(w8, a, srule))) {
                            std::printf("FILTER REJECTED A SHIFTED SELECTION D=%d tau=%g a=%d rule=%d\n", D, tau, a,
                                        srule);
                            return 1;
                        }
                    }
                }
        }
    }
    std::printf("D=%d selected=%ld passed=%ld passed with 16-bit folded words=%ld, 8-bit=%ld\n", D, selected, passed,
                folded_passed, folded8_passed);
    return 0;
}

static int check_bucket_index(int trials) {
    std::vector<long long> bs = {0, 1, -1, 30, 31, 32, -30, -31, -32};
    const long long top = (1LL << 51) - 1;
    for (long long k = -3; k <= 3; ++k) {
        bs.push_back(top + k - 3);
        bs.push_back(-top - k + 3);
    }
    for (int e = 1; e < 51; ++e)
        for (long long k = -2; k <= 2; ++k) {
            bs.push_back((1LL << e) + k);
            bs.push_back(-(1LL << e) + k);
            // multiples of 31 near 2^e
            const long long q = ((1LL << e) / 31) * 31;
            bs.push_back(q + k);
            bs.push_back(-q + k);
        }
    for (int i = 0; i < trials * 10; ++i) {
        const int e = 1 + static_cast<int>(rng() % 50);
        long long v = static_cast<long long>(rng() & ((1ULL << e) - 1));
        bs.push_back(rng() & 1 ? v : -v);
    }
    for (long long b : bs) {
        if (b > top || b < -top) continue;
        const unsigned want = static_cast<unsigned>(((b % 31) + 31) % 31);
        const unsigned got = bucket_index(static_cast<double>(b));
        if (got != want) {
            std::printf("bucket_index(%lld) = %u, want %u\n", b, got, want);
            return 1;
        }
    }
    if (bucket_index(-0.0) != 0u) { std::printf("bucket_index(-0.0)\n"); return 1; }
    return 0;
}

int main(int argc, char** argv) {
    const int trials = argc > 1 ? std::atoi(argv[1]) : 20000;
    int bad = check_bucket_index(trials);
    bad |= check_counts<2>(trials) | check_counts<3>(trials) | check_counts<5>(trials);
    bad |= check_counts<7>(trials) | check_counts<9>(trials) | check_counts<12>(trials);
    bad |= check_counts<16>(trials) | check_counts<20>(trials);
    bad |= check_exactness<3>(trials) | check_exactness<5>(trials) | check_exactness<7>(trials);
    bad |= check_exactness<9>(trials) | check_exactness<13>(trials) | check_exactness<20>(trials / 4);
    if (bad) return 1;
    std::printf("OK\n");
    return 0;
}
