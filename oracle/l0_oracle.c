/*
 * ORACLE — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 implementation of Serial-l0 and
 * Parallel-l0 (Mendoza-Smith & Tanner, "Expander l0-decoding", Algorithms 1
 * and 2, selection rule eq. (selection_l0) in Section 4).  Only the test
 * suite, the package's smoke check and the benchmark's CPU-baseline leg call
 * it; the GPU decoder shares no code with it.  Built with -O2
 * -ffp-contract=off and no fast-math, so every sum, difference and
 * comparison below is one IEEE-754 binary64 operation in the order written.
 * The plain build is single-threaded; a second build of this same file with
 * OpenMP splits the Parallel-l0 vote's columns over threads (nothing else),
 * which changes no arithmetic: both builds give the same result bit for bit.
 *
 * Input (Definition 2.2): A is the binary adjacency matrix of a left
 * d-regular bipartite graph, so column j has exactly d ones, at d distinct
 * rows.  A column that lists a row twice is not such a matrix and the run is
 * rejected as invalid input, like a row index outside [0, m).
 *
 * Readings of the paper that this file fixes (the paper leaves them open):
 *  - zero test and equality: with tau = tol * max_i |y_i| (or tau = tol in
 *    the absolute mode), an entry v counts as nonzero iff |v| > tau; the
 *    paper's exact equality is tol = 0;
 *  - candidate values: for column j only the nonzero values of r on N(j) are
 *    tried as omega (any other omega leaves every entry of r_N(j) nonzero
 *    when tau = 0, so it cannot decrease ||r||_0);
 *  - one update per column: among the candidates reaching the largest
 *    decrease, the smallest value is taken (Algorithms 1-2 write "for omega
 *    in T"; adding two different values to one entry is not a correction);
 *  - threshold: decreases are integers, so "decrease >= alpha" is
 *    "decrease >= ceil(alpha)";
 *  - r <- y - A x_hat is recomputed from scratch (Algorithm 2, last step):
 *    s_i = sum over ascending columns j with i in N(j) of x_hat_j, starting
 *    from +0.0, then r_i = y_i - s_i;
 *  - "while not converged" stops on ||r||_0 = 0 (CONVERGED), on an empty
 *    update set (STALLED: r no longer changes) or after max_iter residual
 *    updates (MAX_ITER); an iteration is the work between two residual
 *    updates (Definition 3.1).
 * Rule MODE scores a candidate by its frequency in r_N(j) instead of the
 * l0-decrease (parallel-LDDSR, Section 4.3 and Table 2).
 *
 * Shifted rules (Section 4.3.1, Algorithm 3 and Theorem 4.8): at the p-th
 * vote pass (p = 0, 1, ...) column j tries one candidate only, the value of r
 * at its (p mod d)-th neighbour in col_idx order, scored by the l0-decrease
 * (SHIFTED_L0DEC) or its frequency (SHIFTED_MODE); a zero candidate is not
 * tried.  A pass that selects nothing leaves r as it is but the next pass
 * tries other positions, so the run stalls only after d consecutive empty
 * passes.  Readings: p counts vote passes, not residual updates; "the
 * (p mod d)-th element of r_N(j)" is taken in col_idx order.
 *
 * Column-scaled A (Section 4.3.3): optional weights w[n], w_j > 0 and finite,
 * make column j of A hold w_j on its d rows, so y_i sums w_j x_j.  Readings:
 *  - the update that zeroes entry t of r_N(j) is omega = r_t / w_j; entry u
 *    of r - omega a_j is then r_u - r_t in exact arithmetic, and it is
 *    evaluated as such, so a column's scores and its chosen entry t are those
 *    of the unscaled rule on the same r (every rule above), and only the
 *    update becomes fl(r_t / w_j);
 *  - w_j > 0 keeps the order of the candidates (the smallest r_t gives the
 *    smallest omega), so the tie-break is unchanged;
 *  - the residual sums the rounded products fl(w_j x_hat_j), from +0.0 over
 *    ascending columns.
 * Without weights every formula reduces to the unit-weight one bit for bit.
 */
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_RULE_L0DEC = 0, ORC_RULE_MODE = 1, ORC_RULE_SHIFTED_L0DEC = 2, ORC_RULE_SHIFTED_MODE = 3 };
enum { ORC_CONVERGED = 0, ORC_STALLED = 1, ORC_MAX_ITER = 2 };
enum { ORC_TOL_RELATIVE = 0, ORC_TOL_ABSOLUTE = 1 };

static int is_nonzero(double v, double tau) { return fabs(v) > tau; }

/*
 * Score of one column on residual values v[0..d) = r restricted to N(j)
 * (eq. (selection_l0)).  For every nonzero candidate omega = v[t] the
 * l0-decrease is ||r||_0 - ||r - omega a_j||_0; only the d rows of N(j)
 * change, so it is counted on them.  Returns 1 and sets *omega when the best
 * decrease reaches a; *best gets the best score (INT_MIN if no candidate).
 */
static int score_column(int32_t d, const double* v, double tau, int32_t rule, int32_t a,
                        double* omega, int32_t* best) {
    int32_t before = 0;
    for (int32_t u = 0; u < d; ++u) before += is_nonzero(v[u], tau);
    int32_t top = INT_MIN;
    double w = 0.0;
    for (int32_t t = 0; t < d; ++t) {
        if (!is_nonzero(v[t], tau)) continue;
        int32_t after = 0, freq = 0;
        for (int32_t u = 0; u < d; ++u) {
            double diff = v[u] - v[t];
            after += is_nonzero(diff, tau);
            freq += !is_nonzero(diff, tau);
        }
        int32_t score = (rule == ORC_RULE_MODE) ? freq : before - after;
        if (top == INT_MIN || score > top || (score == top && v[t] < w)) {
            top = score;
            w = v[t];
        }
    }
    *best = top;
    *omega = w;
    return top != INT_MIN && top >= a;
}

/*
 * Shifted score of one column: the only candidate is omega = v[t]; it is
 * tried when nonzero, scored as in score_column, and selected when the score
 * reaches a.
 */
static int score_column_shifted(int32_t d, const double* v, int32_t t, double tau, int32_t shifted_rule,
                                int32_t a, double* omega) {
    *omega = 0.0;
    if (!is_nonzero(v[t], tau)) return 0;
    int32_t before = 0, after = 0, freq = 0;
    for (int32_t u = 0; u < d; ++u) {
        before += is_nonzero(v[u], tau);
        double diff = v[u] - v[t];
        after += is_nonzero(diff, tau);
        freq += !is_nonzero(diff, tau);
    }
    int32_t score = (shifted_rule == ORC_RULE_SHIFTED_MODE) ? freq : before - after;
    if (score < a) return 0;
    *omega = v[t];
    return 1;
}

static int weights_ok(int64_t n, const double* w) {
    if (!w) return 1;
    for (int64_t j = 0; j < n; ++j)
        if (!(w[j] > 0.0) || !isfinite(w[j])) return 0;
    return 1;
}

/* Column j of A: d row indices, each in [0, m), no row twice (Definition
 * 2.2: a binary matrix with exactly d ones per column). */
static int column_ok(int32_t m, int32_t d, const int32_t* rows) {
    for (int32_t t = 0; t < d; ++t) {
        if (rows[t] < 0 || rows[t] >= m) return 0;
        for (int32_t u = 0; u < t; ++u)
            if (rows[u] == rows[t]) return 0;
    }
    return 1;
}

static int args_ok(int64_t n, int32_t m, int32_t d, const int32_t* col_idx, const double* y,
                   double alpha, int32_t rule, int32_t max_iter, double tol) {
    if (n < 1 || m < 1 || d < 2 || d > m || !col_idx || !y) return 0;
    if (!(alpha > 1.0) || !(alpha <= (double)d)) return 0;
    if (rule < ORC_RULE_L0DEC || rule > ORC_RULE_SHIFTED_MODE) return 0;
    if (max_iter < 0 || !(tol >= 0.0) || !isfinite(tol)) return 0;
    for (int64_t j = 0; j < n; ++j)
        if (!column_ok(m, d, col_idx + j * d)) return 0;
    for (int32_t i = 0; i < m; ++i)
        if (!isfinite(y[i])) return 0;
    return 1;
}

/* tau = tol * max_i |y_i| (relative, tol_mode 0) or tau = tol (absolute). */
static double zero_threshold(int32_t m, const double* y, double tol, int32_t tol_mode) {
    if (tol_mode == ORC_TOL_ABSOLUTE) return tol;
    double s = 0.0;
    for (int32_t i = 0; i < m; ++i)
        if (fabs(y[i]) > s) s = fabs(y[i]);
    return tol * s;
}

/* r = y - A x, each (A x)_i summed from +0.0 over ascending columns; with
 * weights w (or NULL for unit columns) each term is the rounded w_j x_j. */
void orc_residual(int64_t n, int32_t m, int32_t d, const int32_t* col_idx, const double* y,
                  const double* x, const double* w, double* r) {
    double* s = (double*)calloc((size_t)m, sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        const double term = w ? w[j] * x[j] : x[j];
        for (int32_t t = 0; t < d; ++t) s[col_idx[j * d + t]] += term;
    }
    for (int32_t i = 0; i < m; ++i) r[i] = y[i] - s[i];
    free(s);
}

static int32_t count_nonzero(int32_t m, const double* r, double tau) {
    int32_t c = 0;
    for (int32_t i = 0; i < m; ++i) c += is_nonzero(r[i], tau);
    return c;
}

/*
 * Score every column in cols[0..ncols) on the given residual (absolute
 * threshold tau).  sel[c] = 1 and omega[c] = the update when selected;
 * best[c] = best score.  Used to check a single vote step in isolation.
 */
void orc_score_columns(int64_t ncols, int32_t d, const int32_t* rows, const double* r, double tau,
                       int32_t rule, int32_t a, uint8_t* sel, double* omega, int32_t* best) {
    double* v = (double*)malloc(sizeof(double) * (size_t)d);
    for (int64_t c = 0; c < ncols; ++c) {
        for (int32_t t = 0; t < d; ++t) v[t] = r[rows[c * d + t]];
        sel[c] = (uint8_t)score_column(d, v, tau, rule, a, &omega[c], &best[c]);
        if (!sel[c]) omega[c] = 0.0;
    }
    free(v);
}

/* The shifted vote of one pass: column c tries position t only. */
void orc_score_columns_shifted(int64_t ncols, int32_t d, const int32_t* rows, const double* r, double tau,
                               int32_t shifted_rule, int32_t a, int32_t t, uint8_t* sel, double* omega) {
    double* v = (double*)malloc(sizeof(double) * (size_t)d);
    for (int64_t c = 0; c < ncols; ++c) {
        for (int32_t u = 0; u < d; ++u) v[u] = r[rows[c * d + u]];
        sel[c] = (uint8_t)score_column_shifted(d, v, t, tau, shifted_rule, a, &omega[c]);
    }
    free(v);
}

/*
 * ||r||_0 - ||r - omega a_j||_0 over the whole m-vector, forming r - omega a_j
 * entry by entry (the definition in eq. (selection_l0), used as a pin).
 */
int32_t orc_literal_decrease(int32_t m, int32_t d, const int32_t* rows, const double* r,
                             double omega, double tau) {
    double* q = (double*)malloc(sizeof(double) * (size_t)m);
    memcpy(q, r, sizeof(double) * (size_t)m);
    for (int32_t t = 0; t < d; ++t) q[rows[t]] = r[rows[t]] - omega;
    int32_t dec = count_nonzero(m, r, tau) - count_nonzero(m, q, tau);
    free(q);
    return dec;
}

/*
 * Parallel-l0 (Algorithm 2).  tol_mode 0 takes tau = tol * max_i |y_i|, 1
 * takes tau = tol.  x_init (optional) resumes from a previous
 * estimate; w (optional) gives the column weights of a column-scaled A;
 * x_out[n] receives x_hat.  trace[0..iters] receives ||r||_0 after
 * each residual update (trace[0] for the start), tsize[0..iters) the number
 * of columns updated in each iteration; both need max_iter+1 / max_iter
 * slots.  Returns 0, or -1 on invalid arguments.
 */
int orc_parallel_l0(int64_t n, int32_t m, int32_t d, const int32_t* col_idx, const double* y,
                    double alpha, int32_t rule, int32_t max_iter, double tol, int32_t tol_mode,
                    const double* x_init,
                    const double* w, double* x_out, int32_t* trace, int64_t* tsize, int32_t* iters,
                    int32_t* outcome, int32_t* passes) {
    if (!args_ok(n, m, d, col_idx, y, alpha, rule, max_iter, tol) || !weights_ok(n, w) || !x_out ||
        !trace || !iters || !outcome || (tol_mode != ORC_TOL_RELATIVE && tol_mode != ORC_TOL_ABSOLUTE))
        return -1;
    const int32_t a = (int32_t)ceil(alpha);
    const double tau = zero_threshold(m, y, tol, tol_mode);
    double* r = (double*)malloc(sizeof(double) * (size_t)m);
    double* omega = (double*)malloc(sizeof(double) * (size_t)n);
    uint8_t* sel = (uint8_t*)malloc((size_t)n);

    for (int64_t j = 0; j < n; ++j) x_out[j] = x_init ? x_init[j] : 0.0;
    orc_residual(n, m, d, col_idx, y, x_out, w, r);
    const int shifted = rule == ORC_RULE_SHIFTED_L0DEC || rule == ORC_RULE_SHIFTED_MODE;
    int32_t l = 0, p = 0, empty = 0;
    trace[0] = count_nonzero(m, r, tau);
    for (;;) {
        if (trace[l] == 0) { *outcome = ORC_CONVERGED; break; }
        if (l == max_iter) { *outcome = ORC_MAX_ITER; break; }
        /* every column is scored on the same residual; no column's score
           depends on another's, so a build with OpenMP may split the columns
           over threads (each with a gather buffer of its own) and gets the
           same selections bit for bit */
        int64_t chosen = 0;
#pragma omp parallel reduction(+ : chosen)
        {
            double* vt = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
            for (int64_t j = 0; j < n; ++j) {
                int32_t best;
                for (int32_t t = 0; t < d; ++t) vt[t] = r[col_idx[j * d + t]];
                if (shifted)
                    sel[j] = (uint8_t)score_column_shifted(d, vt, p % d, tau, rule, a, &omega[j]);
                else
                    sel[j] = (uint8_t)score_column(d, vt, tau, rule, a, &omega[j], &best);
                chosen += sel[j];
            }
            free(vt);
        }
        ++p;
        if (chosen == 0) {
            /* shifted: r is unchanged, but the next pass tries the next position */
            if (shifted && ++empty < d) continue;
            *outcome = ORC_STALLED;
            break;
        }
        empty = 0;
        /* omega[j] is the residual value the update cancels; on a scaled
           column the update itself is that value over w_j */
        for (int64_t j = 0; j < n; ++j)
            if (sel[j]) x_out[j] = x_out[j] + (w ? omega[j] / w[j] : omega[j]);
        orc_residual(n, m, d, col_idx, y, x_out, w, r);
        if (tsize) tsize[l] = chosen;
        ++l;
        trace[l] = count_nonzero(m, r, tau);
    }
    *iters = l;
    if (passes) *passes = p;
    free(r); free(omega); free(sel);
    return 0;
}

/*
 * Serial-l0 (Algorithm 1): columns are visited in ascending order, each scored
 * on the current residual; a selected column takes its single best update and
 * the d residual entries on N(j) are recomputed at once (each from +0.0 over
 * the ascending columns of its row).  A sweep is one pass over all n
 * columns.  *updates counts residual updates (the paper's iterations),
 * *sweeps the passes; the run stops when ||r||_0 = 0 at the start of a sweep
 * (CONVERGED), after a sweep without updates (STALLED) or after max_sweeps
 * sweeps (MAX_ITER).  Returns 0, or -1 on invalid arguments.
 */
int orc_serial_l0(int64_t n, int32_t m, int32_t d, const int32_t* col_idx, const double* y,
                  double alpha, int32_t rule, int32_t max_sweeps, double tol, double* x_out,
                  int64_t* updates, int32_t* sweeps, int32_t* outcome, int32_t* final_nnz) {
    if (!args_ok(n, m, d, col_idx, y, alpha, rule, max_sweeps, tol) || !x_out || !updates ||
        !sweeps || !outcome || rule > ORC_RULE_MODE)
        return -1;
    const int32_t a = (int32_t)ceil(alpha);
    const double tau = zero_threshold(m, y, tol, ORC_TOL_RELATIVE);
    /* rows of A as ascending column lists (a counting sort over columns) */
    int64_t* rowptr = (int64_t*)calloc((size_t)m + 1, sizeof(int64_t));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    int64_t* rowcol = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n * d));
    for (int64_t e = 0; e < n * (int64_t)d; ++e) rowptr[col_idx[e] + 1]++;
    for (int32_t i = 0; i < m; ++i) rowptr[i + 1] += rowptr[i];
    for (int32_t i = 0; i < m; ++i) fill[i] = rowptr[i];
    for (int64_t j = 0; j < n; ++j)
        for (int32_t t = 0; t < d; ++t) rowcol[fill[col_idx[j * d + t]]++] = j;

    double* r = (double*)malloc(sizeof(double) * (size_t)m);
    double* v = (double*)malloc(sizeof(double) * (size_t)d);
    for (int64_t j = 0; j < n; ++j) x_out[j] = 0.0;
    for (int32_t i = 0; i < m; ++i) r[i] = y[i];
    int64_t upd = 0;
    int32_t sw = 0;
    for (;;) {
        if (count_nonzero(m, r, tau) == 0) { *outcome = ORC_CONVERGED; break; }
        if (sw == max_sweeps) { *outcome = ORC_MAX_ITER; break; }
        int any = 0;
        for (int64_t j = 0; j < n; ++j) {
            double w;
            int32_t best;
            for (int32_t t = 0; t < d; ++t) v[t] = r[col_idx[j * d + t]];
            if (!score_column(d, v, tau, rule, a, &w, &best)) continue;
            x_out[j] = x_out[j] + w;
            ++upd;
            any = 1;
            for (int32_t t = 0; t < d; ++t) {
                int32_t i = col_idx[j * d + t];
                double s = 0.0;
                for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s += x_out[rowcol[p]];
                r[i] = y[i] - s;
            }
        }
        ++sw;
        if (!any) { *outcome = ORC_STALLED; break; }
    }
    *updates = upd;
    *sweeps = sw;
    if (final_nnz) *final_nnz = count_nonzero(m, r, tau);
    free(rowptr); free(fill); free(rowcol); free(r); free(v);
    return 0;
}
