/*
 * Host driver for the sanitizer build of the CPU test infrastructure: draws
 * instances with the generator (every entry point) and runs the oracle's
 * decoders on them (every rule, column weights, a resumed run, Serial-l0,
 * the single-column scorers and the literal decrease), plus the inputs the
 * oracle must refuse.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitize.py; exit status 0 and
 * "OK" when every call behaved.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int l0gen_columns(uint64_t seed, int64_t n, int32_t m, int32_t d, int32_t* col_idx);
int l0gen_support(uint64_t seed, int64_t n, int64_t k, int64_t* supp);
int l0gen_values(uint64_t seed, int64_t k, const int64_t* supp, int32_t kind, double* vals);
int l0gen_weights(uint64_t seed, int64_t n, double lo, double hi, double* w);
int l0gen_measure(int64_t n, int32_t m, int32_t d, const int32_t* col_idx, int64_t k, const int64_t* supp,
                  const double* vals, const double* w, double* y);
void orc_residual(int64_t n, int32_t m, int32_t d, const int32_t* col_idx, const double* y, const double* x,
                  const double* w, double* r);
void orc_score_columns(int64_t ncols, int32_t d, const int32_t* rows, const double* r, double tau, int32_t rule,
                       int32_t a, uint8_t* sel, double* omega, int32_t* best);
void orc_score_columns_shifted(int64_t ncols, int32_t d, const int32_t* rows, const double* r, double tau,
                               int32_t shifted_rule, int32_t a, int32_t t, uint8_t* sel, double* omega);
int32_t orc_literal_decrease(int32_t m, int32_t d, const int32_t* rows, const double* r, double omega, double tau);
int orc_parallel_l0(int64_t n, int32_t m, int32_t d, const int32_t* col_idx, const double* y, double alpha,
                    int32_t rule, int32_t max_iter, double tol, int32_t tol_mode, const double* x_init,
                    const double* w, double* x_out, int32_t* trace, int64_t* tsize, int32_t* iters,
                    int32_t* outcome, int32_t* passes);
int orc_serial_l0(int64_t n, int32_t m, int32_t d, const int32_t* col_idx, const double* y, double alpha,
                  int32_t rule, int32_t max_sweeps, double tol, double* x_out, int64_t* updates, int32_t* sweeps,
                  int32_t* outcome, int32_t* final_nnz);

static int fail(const char* what) {
    printf("FAILED: %s\n", what);
    return 1;
}

/* One instance: every decoder call on it.  Returns 0 on success. */
static int run_instance(uint64_t seed, int64_t n, int32_t m, int32_t d, int64_t k, int kind, int scaled) {
    int32_t* col = malloc(sizeof(int32_t) * (size_t)(n * d));
    int64_t* supp = malloc(sizeof(int64_t) * (size_t)(k ? k : 1));
    double* vals = malloc(sizeof(double) * (size_t)(k ? k : 1));
    double* w = scaled ? malloc(sizeof(double) * (size_t)n) : NULL;
    double* y = malloc(sizeof(double) * (size_t)m);
    double* x = malloc(sizeof(double) * (size_t)n);
    double* x2 = malloc(sizeof(double) * (size_t)n);
    double* r = malloc(sizeof(double) * (size_t)m);
    const int32_t max_iter = 40;
    int32_t* trace = malloc(sizeof(int32_t) * (max_iter + 1));
    int64_t* tsize = malloc(sizeof(int64_t) * max_iter);
    uint8_t* sel = malloc((size_t)n);
    double* om = malloc(sizeof(double) * (size_t)n);
    int32_t* best = malloc(sizeof(int32_t) * (size_t)n);
    int bad = 0;
    if (l0gen_columns(seed, n, m, d, col) || l0gen_support(seed, n, k, supp) ||
        l0gen_values(seed, k, supp, kind, vals) || (w && l0gen_weights(seed, n, 0.5, 1.5, w)) ||
        l0gen_measure(n, m, d, col, k, supp, vals, w, y))
        bad |= fail("generator");
    const double alpha = d >= 4 ? ceil(d / 2.0) : 2.0;
    for (int32_t rule = 0; rule < 4 && !bad; ++rule) {
        int32_t iters, outcome, passes;
        if (orc_parallel_l0(n, m, d, col, y, alpha, rule, max_iter, 1e-10, 0, NULL, w, x, trace, tsize, &iters,
                            &outcome, &passes))
            bad |= fail("parallel");
        /* resume from the result, absolute tolerance */
        if (!bad && orc_parallel_l0(n, m, d, col, y, 2.0, rule, 3, 1e-12, 1, x, w, x2, trace, tsize, &iters,
                                    &outcome, &passes))
            bad |= fail("parallel resume");
    }
    if (!bad) {
        int64_t upd;
        int32_t sweeps, outcome, nnz;
        for (int32_t rule = 0; rule < 2 && !bad; ++rule)
            if (orc_serial_l0(n, m, d, col, y, alpha, rule, 10, 1e-10, x, &upd, &sweeps, &outcome, &nnz))
                bad |= fail("serial");
        orc_residual(n, m, d, col, y, x, w, r);
        orc_score_columns(n, d, col, r, 1e-9, 0, (int32_t)alpha, sel, om, best);
        orc_score_columns_shifted(n, d, col, r, 1e-9, 2, 2, (int32_t)(seed % (uint64_t)d), sel, om);
        (void)orc_literal_decrease(m, d, col, r, r[col[0]], 1e-9);
    }
    /* inputs the oracle must refuse: a repeated row, an index out of range */
    if (!bad) {
        int32_t iters, outcome, passes;
        const int32_t keep = col[d - 1];
        col[d - 1] = col[0];
        if (orc_parallel_l0(n, m, d, col, y, alpha, 0, 5, 1e-10, 0, NULL, w, x, trace, tsize, &iters, &outcome,
                            &passes) != -1)
            bad |= fail("repeated row accepted");
        col[d - 1] = m;
        if (orc_parallel_l0(n, m, d, col, y, alpha, 0, 5, 1e-10, 0, NULL, w, x, trace, tsize, &iters, &outcome,
                            &passes) != -1)
            bad |= fail("row out of range accepted");
        col[d - 1] = keep;
    }
    free(col); free(supp); free(vals); free(w); free(y); free(x); free(x2); free(r);
    free(trace); free(tsize); free(sel); free(om); free(best);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= run_instance(11, 3000, 300, 7, 25, 0, 0);
    bad |= run_instance(12, 2000, 400, 5, 60, 1, 1);
    bad |= run_instance(13, 500, 40, 20, 3, 0, 0);
    bad |= run_instance(14, 1, 3, 2, 1, 0, 0);
    bad |= run_instance(15, 4096, 512, 9, 0, 0, 1);
    bad |= run_instance(16, 257, 60, 3, 10, 1, 0);
    if (bad) return 1;
    printf("OK\n");
    return 0;
}
