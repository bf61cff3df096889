/*
 * mjp_oracle.c -- plain, slow, FP64 CPU reference for the R-MJP expansion.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source with the HIP path.
 *
 * What it computes (Pessoa, Schweiger, Presse, "Avoiding matrix exponentials
 * for large transition rate matrices"):
 *
 *   - the generator A_theta of a reaction network from its rates
 *     (Sec. 2.1.1, Eq. A_def; birth-death Eq. BD_def; the two-species cascade
 *     is the two-index analogue used for the larger workloads);
 *   - Omega = 1.1 max_n |a_nn| and B = I + A/Omega (Eq. B_def);
 *   - the truncated Poisson series of Algorithm 2 (R-MJP, Sec. 2.2.3,
 *     Eq. R-MJP_expansion): rho* = sum_{k=0..K} w_k rho(0) B^k followed by the
 *     residual (1 - sum w_k) placed on the last iterate rho(0) B^K;
 *   - the snapshot log-likelihood sum_i log rho(T^i)_{s^i} (Sec. 2.1.2).
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - Algorithm 2 starts its weight recurrence at exp(-Omega t), which is 0 in
 *     FP64 once Omega t > 745.  The weights are therefore formed in log space,
 *     log w_k = -W + k log W - lgamma(k+1): the same numbers the recurrence
 *     would give with unbounded exponent range.
 *   - The loop "while k <= k*" with the increment first runs floor(k*)+1
 *     products, so the paper's rule gives K = floor(W + 6 sqrt W) + 1.
 *   - The tolerance rule picks the smallest K whose right Poisson tail is at
 *     most eps_right; the series is always accumulated from k = 0 here (the
 *     paper never truncates on the left).
 *   - Truncation of the state space is conservative by default: a transition
 *     that would leave the grid is dropped, so rows of A sum to 0 and rows of
 *     B sum to 1 as Eq. B_def states.  The leaky reading (the exit rate still
 *     counts the dropped transition, as in the m_theta of the birth-death
 *     example) is available as an option.
 *
 * All arithmetic is FP64.  Vector sums use Neumaier compensation so the
 * oracle's own rounding stays near 1e-15 relative.  Row loops are parallel
 * with OpenMP; every output element is still computed by one thread in a fixed
 * order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_BD = 0, ORC_CASCADE2 = 1, ORC_TWOSTATE = 2, ORC_AUTOREG = 3 };
enum { ORC_K_TOL = 0, ORC_K_PAPER = 1 };

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Model generators (Eq. A_def with the model rates).                         */
/* Row index = from-state n, column = to-state m, a_nm = lambda_nm for n != m, */
/* a_nn = -(sum of the rates out of n).                                       */
/* ------------------------------------------------------------------------ */

/* Number of states and an upper bound on the stored entries. */
int orc_model_size(int model, const int32_t* dims, int64_t* n_states, int64_t* nnz_max) {
    if (model == ORC_BD) {
        if (dims[0] < 1) return -1;
        *n_states = dims[0];
        *nnz_max = 3 * (int64_t)dims[0];
        return 0;
    }
    if (model == ORC_CASCADE2) {
        if (dims[0] < 1 || dims[1] < 1) return -1;
        *n_states = (int64_t)dims[0] * dims[1];
        *nnz_max = 5 * *n_states;
        return 0;
    }
    if (model == ORC_TWOSTATE) {
        if (dims[0] < 1) return -1;
        *n_states = 2 * (int64_t)dims[0];
        *nnz_max = 5 * *n_states;
        return 0;
    }
    if (model == ORC_AUTOREG) {
        if (dims[0] < 1 || dims[1] < 1) return -1;
        *n_states = 2 * (int64_t)dims[0] * dims[1];
        *nnz_max = 7 * *n_states;
        return 0;
    }
    return -1;
}

/* One row of a generator from a list of (target, rate) moves out of state
 * n: rates into states off the grid (target < 0) are dropped, or counted in
 * the exit rate only when leaky; zero rates are not stored; entries are
 * emitted in increasing column order with the diagonal -(sum of exits). */
typedef struct { int64_t to; double rate; } orc_move;

static int64_t emit_row(int64_t n, orc_move* mv, int nm, int leaky, int64_t e, int32_t* col, double* val) {
    double out = 0.0;
    for (int i = 0; i < nm; ++i)
        if (mv[i].rate != 0.0 && (mv[i].to >= 0 || leaky)) out += mv[i].rate;
    /* insertion sort of the kept moves by target, with the diagonal */
    orc_move kept[8];
    int nk = 0;
    for (int i = 0; i < nm; ++i)
        if (mv[i].rate != 0.0 && mv[i].to >= 0) kept[nk++] = mv[i];
    kept[nk].to = n;
    kept[nk].rate = -out;
    ++nk;
    for (int i = 1; i < nk; ++i)
        for (int j = i; j > 0 && kept[j - 1].to > kept[j].to; --j) {
            orc_move t = kept[j]; kept[j] = kept[j - 1]; kept[j - 1] = t;
        }
    for (int i = 0; i < nk; ++i) { col[e] = (int32_t)kept[i].to; val[e] = kept[i].rate; ++e; }
    return e;
}

/*
 * Fill the generator in CSR form.  Structural zeros (a zero rate) are not
 * stored.  Returns the number of stored entries, or -1 on bad input.
 *
 * Birth-death (Eq. BD_def): theta = (beta, gamma); n -> n+1 at beta,
 * n -> n-1 at gamma*n.
 *
 * Two-species cascade on an S1 x S2 grid, state index n = n1 + S1*n2 (first
 * coordinate fastest, the convention of the paper's multi-index examples):
 * theta = (k1, g1, k2, g2);  (n1,n2)->(n1+1,n2) at k1, ->(n1-1,n2) at g1*n1,
 * ->(n1,n2+1) at k2*n1, ->(n1,n2-1) at g2*n2.
 */
int64_t orc_model_generator(int model, const double* theta, const int32_t* dims, int leaky,
                            int64_t* row_ptr, int32_t* col, double* val) {
    int64_t e = 0;
    if (model == ORC_BD) {
        const double beta = theta[0], gamma = theta[1];
        const int32_t N = dims[0];
        for (int32_t n = 0; n < N; ++n) {
            row_ptr[n] = e;
            double out = 0.0;
            const double death = gamma * (double)n;
            const double birth = beta;
            if (n >= 1 && death != 0.0) out += death;
            if (n + 1 < N && birth != 0.0) out += birth;
            else if (leaky) out += birth;
            if (n >= 1 && death != 0.0) { col[e] = n - 1; val[e] = death; ++e; }
            col[e] = n; val[e] = -out; ++e;
            if (n + 1 < N && birth != 0.0) { col[e] = n + 1; val[e] = birth; ++e; }
        }
        row_ptr[N] = e;
        return e;
    }
    if (model == ORC_CASCADE2) {
        const double k1 = theta[0], g1 = theta[1], k2 = theta[2], g2 = theta[3];
        const int32_t S1 = dims[0], S2 = dims[1];
        for (int32_t n2 = 0; n2 < S2; ++n2) {
            for (int32_t n1 = 0; n1 < S1; ++n1) {
                const int64_t n = (int64_t)n1 + (int64_t)S1 * n2;
                row_ptr[n] = e;
                const double r_b1 = k1;                 /* to (n1+1, n2) */
                const double r_d1 = g1 * (double)n1;    /* to (n1-1, n2) */
                const double r_b2 = k2 * (double)n1;    /* to (n1, n2+1) */
                const double r_d2 = g2 * (double)n2;    /* to (n1, n2-1) */
                const int in_b1 = (n1 + 1 < S1), in_b2 = (n2 + 1 < S2);
                double out = 0.0;
                if (r_d2 != 0.0 && n2 >= 1) out += r_d2;
                if (r_d1 != 0.0 && n1 >= 1) out += r_d1;
                if (in_b1 || leaky) out += r_b1;
                if (in_b2 || leaky) out += r_b2;
                if (n2 >= 1 && r_d2 != 0.0) { col[e] = (int32_t)(n - S1); val[e] = r_d2; ++e; }
                if (n1 >= 1 && r_d1 != 0.0) { col[e] = (int32_t)(n - 1); val[e] = r_d1; ++e; }
                col[e] = (int32_t)n; val[e] = -out; ++e;
                if (in_b1 && r_b1 != 0.0) { col[e] = (int32_t)(n + 1); val[e] = r_b1; ++e; }
                if (in_b2 && r_b2 != 0.0) { col[e] = (int32_t)(n + S1); val[e] = r_b2; ++e; }
            }
        }
        row_ptr[(int64_t)S1 * S2] = e;
        return e;
    }
    if (model == ORC_TWOSTATE) {
        /* Two-state birth-death (Sec. 3.1.2, Eq. 2S_chem): theta = (beta, gamma,
         * lambda_act, lambda_ina); state n = n_R + s N_R with s = 0 active,
         * s = 1 inactive.  Active: n_R -> n_R+1 at beta.  Both: n_R -> n_R-1 at
         * gamma n_R.  Active -> inactive at lambda_ina, inactive -> active at
         * lambda_act (the text's labels; births never wrap into the other gene
         * state). */
        const double beta = theta[0], gamma = theta[1], lact = theta[2], lina = theta[3];
        const int32_t NR = dims[0];
        for (int32_t s = 0; s < 2; ++s)
            for (int32_t r = 0; r < NR; ++r) {
                const int64_t n = r + (int64_t)s * NR;
                row_ptr[n] = e;
                orc_move mv[4];
                int nm = 0;
                if (s == 0) { mv[nm].to = (r + 1 < NR) ? n + 1 : -1; mv[nm].rate = beta; ++nm; }
                if (r >= 1) { mv[nm].to = n - 1; mv[nm].rate = gamma * (double)r; ++nm; }
                if (s == 0) { mv[nm].to = n + NR; mv[nm].rate = lina; ++nm; }
                else { mv[nm].to = n - NR; mv[nm].rate = lact; ++nm; }
                e = emit_row(n, mv, nm, leaky, e, col, val);
            }
        row_ptr[2 * (int64_t)NR] = e;
        return e;
    }
    if (model == ORC_AUTOREG) {
        /* Autoregulatory gene network (Sec. 3.1.3, Eq. STS_chem): theta =
         * (beta_R, beta_P, gamma_R, gamma_P, lambda_act, lambda_ina); state
         * n = n_R + n_P N_R + s N_R N_P (s = 0 active, 1 inactive), N = 2 N_R N_P.
         * Active: R born at beta_R.  Any: P born at beta_P n_R; R dies at
         * gamma_R n_R; P dies at gamma_P n_P.  Active + P -> inactive at
         * lambda_ina n_P (one P bound); inactive -> active + P at lambda_act. */
        const double bR = theta[0], bP = theta[1], gR = theta[2], gP = theta[3], lact = theta[4], lina = theta[5];
        const int32_t NR = dims[0], NP = dims[1];
        const int64_t plane = (int64_t)NR * NP;
        for (int32_t s = 0; s < 2; ++s)
            for (int32_t p = 0; p < NP; ++p)
                for (int32_t r = 0; r < NR; ++r) {
                    const int64_t n = r + (int64_t)p * NR + s * plane;
                    row_ptr[n] = e;
                    orc_move mv[6];
                    int nm = 0;
                    if (s == 0) { mv[nm].to = (r + 1 < NR) ? n + 1 : -1; mv[nm].rate = bR; ++nm; }
                    mv[nm].to = (p + 1 < NP) ? n + NR : -1; mv[nm].rate = bP * (double)r; ++nm;
                    if (r >= 1) { mv[nm].to = n - 1; mv[nm].rate = gR * (double)r; ++nm; }
                    if (p >= 1) { mv[nm].to = n - NR; mv[nm].rate = gP * (double)p; ++nm; }
                    if (s == 0 && p >= 1) { mv[nm].to = n + plane - NR; mv[nm].rate = lina * (double)p; ++nm; }
                    if (s == 1) { mv[nm].to = (p + 1 < NP) ? n - plane + NR : -1; mv[nm].rate = lact; ++nm; }
                    e = emit_row(n, mv, nm, leaky, e, col, val);
                }
        row_ptr[2 * plane] = e;
        return e;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Poisson weights (Eq. ME_uniform; Algorithm 2's P_Poisson).                 */
/* ------------------------------------------------------------------------ */

static double log_pois(int64_t k, double W) {
    if (W == 0.0) return k == 0 ? 0.0 : -INFINITY;
    return -W + (double)k * log(W) - lgamma((double)k + 1.0);
}

double orc_poisson_logpmf(int64_t k, double W) { return log_pois(k, W); }

/* Upper index beyond which the Poisson(W) mass is far below 1e-300. */
static int64_t far_right(double W) {
    return (int64_t)ceil(W + 40.0 * sqrt(W) + 200.0);
}

/*
 * Jump count K.
 *   paper rule (Algorithm 2's loop bound): K = floor(W + 6 sqrt W) + 1;
 *   tolerance rule: the smallest K with sum_{j>K} w_j <= eps_right.
 * The right tail is summed from far out towards the mode, smallest terms
 * first.  Returns K, and the right tail mass in *tail_out.
 */
int64_t orc_pick_K(double W, int k_rule, double eps_right, double* tail_out) {
    int64_t K;
    if (W <= 0.0) { if (tail_out) *tail_out = 0.0; return 0; }
    if (k_rule == ORC_K_PAPER) {
        K = (int64_t)floor(W + 6.0 * sqrt(W)) + 1;
    } else {
        const int64_t hi = far_right(W);
        double tail = 0.0;
        K = 0;
        for (int64_t j = hi; j >= 1; --j) {
            /* tail currently holds sum_{i > j} w_i */
            const double next = tail + exp(log_pois(j, W));
            if (next > eps_right) { K = j; break; }
            tail = next;
        }
    }
    if (tail_out) {
        double tail = 0.0;
        const int64_t hi = far_right(W) > K ? far_right(W) : K + 1;
        for (int64_t j = hi; j > K; --j) tail += exp(log_pois(j, W));
        *tail_out = tail;
    }
    return K;
}

/* w_k for k = 0..K into w[0..K]; returns sum_{k<=K} w_k (Neumaier sum). */
double orc_weights(double W, int64_t K, double* w) {
    double s = 0.0, c = 0.0;
    for (int64_t k = 0; k <= K; ++k) {
        const double x = exp(log_pois(k, W));
        w[k] = x;
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x; else c += (x - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------------ */
/* Expansion (Algorithm 2).                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    double omega;       /* Omega = factor * max_n |a_nn| (Eq. B_def) */
    double W;           /* Omega * t */
    double eps_right;   /* sum_{k>K} w_k */
    double residual;    /* 1 - sum_{k<=K} w_k, lumped onto rho(0) B^K */
    double mass_in;     /* sum of rho(0) */
    double mass_out;    /* sum of the result */
    int64_t K;          /* number of products rho <- rho B */
} orc_info;

/* Transpose the CSR pattern of B = I + A/Omega: row m of the result lists the
 * entries b_nm of column m of B (the pull form of the row-vector product). */
static void build_pull(int64_t n, const int64_t* rp, const int32_t* ci, const double* a, double omega,
                       int64_t* trp, int32_t* tci, double* tb) {
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t r = 0; r < n; ++r)
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) cnt[ci[e] + 1]++;
    trp[0] = 0;
    for (int64_t m = 0; m < n; ++m) trp[m + 1] = trp[m] + cnt[m + 1];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t m = 0; m < n; ++m) fill[m] = trp[m];
    for (int64_t r = 0; r < n; ++r) {
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t m = ci[e];
            const double b = (m == r ? 1.0 : 0.0) + a[e] / omega;  /* Eq. B_def */
            tci[fill[m]] = (int32_t)r;
            tb[fill[m]] = b;
            fill[m]++;
        }
    }
    free(fill);
    free(cnt);
}

static double max_abs_diag(int64_t n, const int64_t* rp, const int32_t* ci, const double* a) {
    double m = 0.0;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e)
            if (ci[e] == r && fabs(a[e]) > m) m = fabs(a[e]);
    return m;
}

static double vec_sum(int64_t n, const double* x) {
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) c += (s - t) + x[i]; else c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}

/* acc (sum, comp) += a * x, Neumaier per element */
static void acc_axpy(int64_t n, double a, const double* x, double* s, double* c) {
    if (a == 0.0) return;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double v = a * x[i];
        const double t = s[i] + v;
        if (fabs(s[i]) >= fabs(v)) c[i] += (s[i] - t) + v; else c[i] += (v - t) + s[i];
        s[i] = t;
    }
}

/*
 * rho_out = R-MJP approximation of rho0 * exp(A t) (Algorithm 2).
 *   omega_factor: Omega = omega_factor * max_n |a_nn| (the paper uses 1.1);
 *   k_rule / eps_right: how K is chosen (see orc_pick_K);
 *   lump: 1 adds the residual (1 - sum_{k<=K} w_k) times rho0 B^K, as the last
 *         line of Algorithm 2 does; 0 leaves it out.
 * Special cases: t == 0 or an all-zero diagonal (Omega == 0) return rho0.
 * Returns 0, or -1 on bad input.
 */
int orc_expv(int64_t n, const int64_t* rp, const int32_t* ci, const double* a, const double* rho0,
             double t, double omega_factor, int k_rule, double eps_right, int lump,
             double* rho_out, orc_info* info) {
    if (n < 1 || t < 0.0 || !(omega_factor > 1.0)) return -1;
    orc_info loc;
    memset(&loc, 0, sizeof loc);
    loc.mass_in = vec_sum(n, rho0);
    const double m_theta = max_abs_diag(n, rp, ci, a);
    if (t == 0.0 || m_theta == 0.0) {
        memcpy(rho_out, rho0, sizeof(double) * (size_t)n);
        loc.mass_out = loc.mass_in;
        if (info) *info = loc;
        return 0;
    }
    const double omega = omega_factor * m_theta;
    const double W = omega * t;
    double tail = 0.0;
    const int64_t K = orc_pick_K(W, k_rule, eps_right, &tail);
    double* w = (double*)malloc(sizeof(double) * (size_t)(K + 1));
    const double pc = orc_weights(W, K, w);            /* P_Cumulative */

    const int64_t nnz = rp[n];
    int64_t* trp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* tci = (int32_t*)malloc(sizeof(int32_t) * (size_t)nnz);
    double* tb = (double*)malloc(sizeof(double) * (size_t)nnz);
    build_pull(n, rp, ci, a, omega, trp, tci, tb);

    double* cur = (double*)malloc(sizeof(double) * (size_t)n);
    double* nxt = (double*)malloc(sizeof(double) * (size_t)n);
    double* s = (double*)calloc((size_t)n, sizeof(double));
    double* c = (double*)calloc((size_t)n, sizeof(double));
    memcpy(cur, rho0, sizeof(double) * (size_t)n);
    acc_axpy(n, w[0], cur, s, c);                      /* rho* = P rho */
    for (int64_t k = 1; k <= K; ++k) {
        /* rho <- rho B : new_m = sum_n rho_n b_nm, one output row per m */
        #pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < n; ++m) {
            double acc = 0.0;
            for (int64_t e = trp[m]; e < trp[m + 1]; ++e) acc += cur[tci[e]] * tb[e];
            nxt[m] = acc;
        }
        double* tmp = cur; cur = nxt; nxt = tmp;
        acc_axpy(n, w[k], cur, s, c);                  /* rho* += P rho */
    }
    const double resid = 1.0 - pc;
    if (lump) acc_axpy(n, resid, cur, s, c);           /* rho* += (1 - P_c) rho */
    for (int64_t i = 0; i < n; ++i) rho_out[i] = s[i] + c[i];

    loc.omega = omega;
    loc.W = W;
    loc.eps_right = tail;
    loc.residual = resid;
    loc.K = K;
    loc.mass_out = vec_sum(n, rho_out);
    if (info) *info = loc;
    free(w); free(trp); free(tci); free(tb); free(cur); free(nxt); free(s); free(c);
    return 0;
}

/* One product y = x B (B = I + A/Omega, Omega = omega_factor * max|a_nn|),
 * exposed so a test can compare a single jump with a dense product. */
int orc_jump(int64_t n, const int64_t* rp, const int32_t* ci, const double* a, double omega_factor,
             const double* x, double* y) {
    const double omega = omega_factor * max_abs_diag(n, rp, ci, a);
    if (!(omega > 0.0)) return -1;
    for (int64_t m = 0; m < n; ++m) y[m] = 0.0;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e)
            y[ci[e]] += x[r] * ((ci[e] == r ? 1.0 : 0.0) + a[e] / omega);
    return 0;
}

/*
 * Snapshot log-likelihood (Sec. 2.1.2): sum_i c_i log rho(T_{j_i})_{s_i}.
 * Each collection time gets an independent solve from rho0.  obs holds n_obs
 * triples (time index, state index, count).  A non-positive probability gives
 * -inf.  Returns 0, or -1 on bad input.
 */
int orc_loglik(int64_t n, const int64_t* rp, const int32_t* ci, const double* a, const double* rho0,
               int32_t n_t, const double* T, int32_t n_obs, const int32_t* obs,
               double omega_factor, int k_rule, double eps_right, double* out_ll) {
    double* rho = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n_t);
    for (int32_t j = 0; j < n_t; ++j) {
        if (orc_expv(n, rp, ci, a, rho0, T[j], omega_factor, k_rule, eps_right, 1,
                     rho + (size_t)j * (size_t)n, NULL) != 0) { free(rho); return -1; }
    }
    double s = 0.0, c = 0.0;
    int neg_inf = 0;
    for (int32_t i = 0; i < n_obs; ++i) {
        const int32_t j = obs[3 * i], st = obs[3 * i + 1], cnt = obs[3 * i + 2];
        if (j < 0 || j >= n_t || st < 0 || st >= n) { neg_inf = 1; continue; }
        const double p = rho[(size_t)j * (size_t)n + (size_t)st];
        if (!(p > 0.0)) { neg_inf = 1; continue; }
        const double x = (double)cnt * log(p);
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x; else c += (x - t) + s;
        s = t;
    }
    *out_ll = neg_inf ? -INFINITY : s + c;
    free(rho);
    return 0;
}
