/*
 * Sanitizer driver for the library's host-side validation (test
 * infrastructure): tests/test_sanitizers.py builds the library's host code
 * (no device code) with AddressSanitizer and UndefinedBehaviorSanitizer and
 * links this program against it.  Every call below is rejected, or answered,
 * on the host before any launch: invalid operators and options, null
 * arguments, bad observation records, bad surrogate and sampler
 * configurations, the host-only model generator and counter-based generator,
 * and a valid operator on a machine without a GPU (MJP_E_DEVICE).  Exit
 * status 0 only if every status matches and neither sanitizer reported.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mjp.h"

static int failures = 0;
#define EXPECT(call, want)                                                                  \
    do {                                                                                    \
        const mjp_status got_ = (call);                                                     \
        if (got_ != (want)) {                                                               \
            fprintf(stderr, "FAIL line %d: %s -> %d, want %d (%s)\n", __LINE__, #call, (int)got_, \
                    (int)(want), mjp_last_error());                                         \
            ++failures;                                                                     \
        } else if (got_ != MJP_OK && strlen(mjp_last_error()) == 0) {                       \
            fprintf(stderr, "FAIL line %d: no error message\n", __LINE__);                  \
            ++failures;                                                                     \
        }                                                                                   \
    } while (0)

static mjp_status plan_csr(const int32_t* rp, const int32_t* ci, const double* v, int32_t n, const mjp_opts* o) {
    mjp_csr A = {n, n > 0 ? rp[n] : 0, rp, ci, v};
    mjp_plan* p = NULL;
    const mjp_status st = mjp_plan_create_csr(&A, o, &p);
    if (p) mjp_plan_destroy(p);
    return st;
}

int main(void) {
    const int32_t rp[3] = {0, 2, 4}, ci[4] = {0, 1, 0, 1}, ci_uns[4] = {1, 0, 0, 1}, ci_oob[4] = {0, 2, 0, 1};
    const int32_t rp_bad[3] = {0, 3, 4};
    const double good[4] = {-1.0, 1.0, 2.0, -2.0}, neg[4] = {-1.0, -1.0, 2.0, -2.0};
    const double good_uns[4] = {1.0, -1.0, 2.0, -2.0};  /* the good operator with row 0's entries swapped */
    const double nonzero_sum[4] = {-1.5, 1.0, 2.0, -2.0}, nan_v[4] = {-1.0, NAN, 2.0, -2.0};
    mjp_opts o;
    mjp_opts_default(&o);

    /* operators */
    EXPECT(plan_csr(rp, ci, neg, 2, &o), MJP_E_NOT_GENERATOR);
    EXPECT(plan_csr(rp, ci, nonzero_sum, 2, &o), MJP_E_NOT_GENERATOR);
    EXPECT(plan_csr(rp, ci_uns, good_uns, 2, &o), MJP_E_INVALID_ARG);
    EXPECT(plan_csr(rp, ci_oob, good, 2, &o), MJP_E_INVALID_ARG);
    {
        mjp_csr A = {2, 4, rp_bad, ci, good};
        mjp_plan* p = NULL;
        EXPECT(mjp_plan_create_csr(&A, &o, &p), MJP_E_INVALID_ARG);
    }
    EXPECT(plan_csr(rp, ci, nan_v, 2, &o), MJP_E_INVALID_ARG);
    EXPECT(plan_csr(rp, ci, good, 0, &o), MJP_E_INVALID_ARG);
    EXPECT(mjp_plan_create_csr(NULL, NULL, NULL), MJP_E_INVALID_ARG);
    EXPECT(mjp_plan_create_stencil(NULL, NULL, NULL), MJP_E_INVALID_ARG);

    /* options */
    {
        mjp_opts b = o;
        b.omega_factor = 1.0;
        EXPECT(plan_csr(rp, ci, good, 2, &b), MJP_E_INVALID_ARG);
        b = o;
        b.tol = 1.5;
        EXPECT(plan_csr(rp, ci, good, 2, &b), MJP_E_INVALID_ARG);
        b = o;
        b.reserved[3] = 7;
        EXPECT(plan_csr(rp, ci, good, 2, &b), MJP_E_INVALID_ARG);
    }

    /* models: validation, and the host-only generator (rows sum to zero) */
    {
        mjp_model m;
        memset(&m, 0, sizeof m);
        m.model = 9;
        m.dims[0] = m.dims[1] = 4;
        int32_t n = 0, nnz = 0;
        EXPECT(mjp_model_csr_size(&m, MJP_CONSERVATIVE, &n, &nnz), MJP_E_INVALID_ARG);
        m.model = MJP_MODEL_CASCADE2;
        m.theta[0] = -1.0;
        EXPECT(mjp_model_csr_size(&m, MJP_CONSERVATIVE, &n, &nnz), MJP_E_INVALID_ARG);
        const double th[4] = {20.0, 1.0, 0.5, 0.5};
        memcpy(m.theta, th, sizeof th);
        m.dims[0] = 12;
        m.dims[1] = 7;
        EXPECT(mjp_model_csr_size(&m, MJP_CONSERVATIVE, &n, &nnz), MJP_OK);
        int32_t mrp[12 * 7 + 1], mci[5 * 12 * 7];
        double mv[5 * 12 * 7];
        if (n == 84 && nnz <= 5 * 84) {
            EXPECT(mjp_model_csr(&m, MJP_CONSERVATIVE, mrp, mci, mv), MJP_OK);
            for (int r = 0; r < n; ++r) {
                double s = 0.0;
                for (int q = mrp[r]; q < mrp[r + 1]; ++q) s += mv[q];
                if (fabs(s) > 1e-12) {
                    fprintf(stderr, "FAIL: model row %d sums to %g\n", r, s);
                    ++failures;
                }
            }
        } else {
            fprintf(stderr, "FAIL: model size %d %d\n", n, nnz);
            ++failures;
        }
    }

    /* likelihood records */
    {
        const double T[2] = {1.0, -2.0}, dummy[8] = {0};
        const int32_t rec_ok[4] = {0, 1, 1, 1}, rec_t[4] = {3, 1, 1, 1}, rec_c0[4] = {0, 1, 1, 0};
        const int32_t rec_neg[4] = {0, -1, 1, 1};
        mjp_obs ob = {1, T, 1, rec_ok, {0, 0}};
        double ll[1];
        EXPECT(mjp_loglik(5, 1, dummy, (const int32_t*)dummy, &ob, &o, ll, NULL, NULL), MJP_E_INVALID_ARG);
        EXPECT(mjp_loglik(1, -1, dummy, (const int32_t*)dummy, &ob, &o, ll, NULL, NULL), MJP_E_INVALID_ARG);
        ob.obs_h = rec_t;
        EXPECT(mjp_loglik(1, 1, dummy, (const int32_t*)dummy, &ob, &o, ll, NULL, NULL), MJP_E_INVALID_ARG);
        ob.obs_h = rec_c0;
        EXPECT(mjp_loglik(1, 1, dummy, (const int32_t*)dummy, &ob, &o, ll, NULL, NULL), MJP_E_INVALID_ARG);
        ob.obs_h = rec_neg;
        EXPECT(mjp_loglik(1, 1, dummy, (const int32_t*)dummy, &ob, &o, ll, NULL, NULL), MJP_E_INVALID_ARG);
        ob.obs_h = rec_ok;
        ob.n_t = 2;
        EXPECT(mjp_loglik(1, 1, dummy, (const int32_t*)dummy, &ob, &o, ll, NULL, NULL), MJP_E_INVALID_ARG);
        ob.n_t = 1;
        ob.x0[0] = -1;
        EXPECT(mjp_loglik(1, 1, dummy, (const int32_t*)dummy, &ob, &o, ll, NULL, NULL), MJP_E_INVALID_ARG);
        ob.x0[0] = 0;
        EXPECT(mjp_loglik(1, 0, dummy, (const int32_t*)dummy, &ob, &o, ll, NULL, NULL), MJP_OK);
    }

    /* surrogate and sampler configurations */
    {
        const mjp_mlp_cfg bad[4] = {{0, 256, 3}, {4, 100, 3}, {4, 1024, 3}, {4, 256, 9}};
        for (int i = 0; i < 4; ++i) {
            mjp_surrogate* s = NULL;
            EXPECT(mjp_surrogate_create(&bad[i], 0, &s), MJP_E_INVALID_ARG);
        }
        EXPECT(mjp_surrogate_load(NULL, NULL), MJP_E_INVALID_ARG);
        mjp_sampler_cfg sc;
        mjp_sampler_cfg_default(&sc);
        sc.chains = 0;
        const double T[1] = {1.0};
        const int32_t rec[4] = {0, 1, 1, 1};
        mjp_obs ob = {1, T, 1, rec, {0, 0}};
        mjp_sampler* smp = NULL;
        EXPECT(mjp_sampler_create(&sc, &ob, &o, &smp), MJP_E_INVALID_ARG);
    }

    /* the counter-based generator's host form: deterministic, key-sensitive */
    {
        const uint32_t c[4] = {1, 2, 3, 4}, k[2] = {5, 6}, k2[2] = {5, 7};
        uint32_t a[4], b[4], d[4];
        mjp_philox4x32_10(c, k, a);
        mjp_philox4x32_10(c, k, b);
        mjp_philox4x32_10(c, k2, d);
        if (memcmp(a, b, sizeof a) != 0 || memcmp(a, d, sizeof a) == 0) {
            fprintf(stderr, "FAIL: philox host form\n");
            ++failures;
        }
    }

    /* a valid operator: the host checks pass and the device step is reached */
    {
        const mjp_status st = plan_csr(rp, ci, good, 2, &o);
        if (st != MJP_E_DEVICE && st != MJP_OK) {
            fprintf(stderr, "FAIL: valid operator -> %d (%s)\n", (int)st, mjp_last_error());
            ++failures;
        }
    }
    EXPECT(mjp_shutdown(), MJP_OK);
    if (failures) fprintf(stderr, "%d checks failed\n", failures);
    else printf("abi driver: all checks passed (%s)\n", mjp_version());
    return failures ? 1 : 0;
}
