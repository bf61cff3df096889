/*
 * Sanitizer driver for the FP64 oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py
 * and run on small inputs of every model, including the degenerate cases
 * (t = 0, an all-zero generator, invalid arguments, a far-right Poisson
 * window, observations off the grid).  Exit status 0 only if every check
 * holds and neither sanitizer reported anything.
 */
#include "../../oracle/mjp_oracle.c"

#include <stdio.h>

static int failures = 0;
#define CHECK(c, ...)                         \
    do {                                      \
        if (!(c)) {                           \
            fprintf(stderr, "FAIL: " __VA_ARGS__); \
            fprintf(stderr, "\n");            \
            ++failures;                       \
        }                                     \
    } while (0)

static void run_model(int model, const double* theta, int32_t d0, int32_t d1) {
    const int32_t dims[2] = {d0, d1};
    int64_t n = 0, nnz = 0;
    CHECK(orc_model_size(model, dims, &n, &nnz) == 0 && n > 0 && nnz > 0, "model %d size", model);
    for (int leaky = 0; leaky <= 1; ++leaky) {
        int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int32_t* ci = (int32_t*)malloc(sizeof(int32_t) * (size_t)nnz);
        double* a = (double*)malloc(sizeof(double) * (size_t)nnz);
        const int64_t e = orc_model_generator(model, theta, dims, leaky, rp, ci, a);
        CHECK(e > 0 && e <= nnz && rp[n] == e, "model %d generator entries", model);
        for (int64_t r = 0; r < n && !leaky; ++r) {  /* conservative: rows sum to zero */
            double s = 0.0;
            for (int64_t q = rp[r]; q < rp[r + 1]; ++q) s += a[q];
            CHECK(fabs(s) < 1e-9, "model %d row %lld sums to %g", model, (long long)r, s);
        }
        double* rho0 = (double*)calloc((size_t)n, sizeof(double));
        double* out = (double*)malloc(sizeof(double) * (size_t)n);
        double* y = (double*)malloc(sizeof(double) * (size_t)n);
        rho0[0] = 1.0;
        const double ts[3] = {0.0, 0.5, 3.0};
        for (int k_rule = 0; k_rule <= 1; ++k_rule)
            for (int i = 0; i < 3; ++i) {
                orc_info inf;
                CHECK(orc_expv(n, rp, ci, a, rho0, ts[i], 1.1, k_rule, 1e-12, 1, out, &inf) == 0, "expv");
                double m = 0.0, lo = 0.0;
                for (int64_t r = 0; r < n; ++r) {
                    m += out[r];
                    if (out[r] < lo) lo = out[r];
                }
                if (!leaky) CHECK(fabs(m - 1.0) < 1e-9, "model %d t %g mass %.17g", model, ts[i], m);
                CHECK(lo > -1e-14, "model %d negative entry %g", model, lo);
            }
        CHECK(orc_jump(n, rp, ci, a, 1.1, rho0, y) == 0, "jump");
        CHECK(orc_expv(0, rp, ci, a, rho0, 1.0, 1.1, 0, 1e-9, 1, out, NULL) == -1, "n = 0 accepted");
        CHECK(orc_expv(n, rp, ci, a, rho0, -1.0, 1.1, 0, 1e-9, 1, out, NULL) == -1, "t < 0 accepted");
        CHECK(orc_expv(n, rp, ci, a, rho0, 1.0, 1.0, 0, 1e-9, 1, out, NULL) == -1, "omega factor 1 accepted");
        /* log-likelihood: one record on the grid, one off it (-inf) */
        const double T[2] = {0.5, 1.0};
        const int32_t obs_ok[6] = {0, 0, 2, 1, (int32_t)(n - 1), 1};
        double ll = 0.0;
        CHECK(orc_loglik(n, rp, ci, a, rho0, 2, T, 2, obs_ok, 1.1, 0, 1e-12, &ll) == 0, "loglik");
        CHECK(ll <= 0.0, "loglik %g > 0", ll);
        const int32_t obs_off[3] = {1, (int32_t)n, 1};
        CHECK(orc_loglik(n, rp, ci, a, rho0, 2, T, 1, obs_off, 1.1, 0, 1e-12, &ll) == 0 && isinf(ll) && ll < 0,
              "off-grid record");
        free(rp); free(ci); free(a); free(rho0); free(out); free(y);
    }
}

int main(void) {
    const double bd[2] = {40.0, 1.0}, cas[4] = {20.0, 1.0, 0.5, 0.5};
    const double two[4] = {20.0, 1.0, 0.3, 0.7}, aut[6] = {8.0, 2.0, 1.0, 1.0, 0.2, 0.4};
    run_model(ORC_BD, bd, 80, 1);
    run_model(ORC_CASCADE2, cas, 24, 17);
    run_model(ORC_TWOSTATE, two, 40, 1);
    run_model(ORC_AUTOREG, aut, 12, 9);
    /* an all-zero generator returns rho0 */
    {
        const double z[2] = {0.0, 0.0};
        const int32_t dims[2] = {5, 1};
        int64_t rp[6], n = 0, nnz = 0;
        int32_t ci[16];
        double a[16], rho0[5] = {0.2, 0.2, 0.2, 0.2, 0.2}, out[5];
        CHECK(orc_model_size(ORC_BD, dims, &n, &nnz) == 0 && n == 5 && nnz <= 16, "zero size");
        orc_model_generator(ORC_BD, z, dims, 0, rp, ci, a);
        CHECK(orc_expv(5, rp, ci, a, rho0, 2.0, 1.1, 0, 1e-9, 1, out, NULL) == 0 && out[3] == 0.2, "zero generator");
    }
    /* Poisson windows: tiny, moderate and far-right (log-space weights) */
    const double Ws[4] = {1e-3, 3.0, 900.0, 4.0e4};
    for (int i = 0; i < 4; ++i) {
        double tail = -1.0;
        const int64_t K = orc_pick_K(Ws[i], 0, 1e-12, &tail);
        CHECK(K >= 0 && tail >= 0.0 && tail <= 1e-12, "pick_K W %g", Ws[i]);
        double* w = (double*)malloc(sizeof(double) * (size_t)(K + 1));
        const double pc = orc_weights(Ws[i], K, w);
        CHECK(pc > 1.0 - 1e-9 && pc <= 1.0 + 1e-12, "weights W %g sum %.17g", Ws[i], pc);
        CHECK(isfinite(orc_poisson_logpmf(K, Ws[i])), "logpmf");
        free(w);
        const int64_t Kp = orc_pick_K(Ws[i], 1, 0.0, &tail);
        CHECK(Kp >= 1, "paper rule W %g", Ws[i]);
    }
    if (failures) fprintf(stderr, "%d checks failed\n", failures);
    else printf("oracle driver: all checks passed\n");
    return failures ? 1 : 0;
}
