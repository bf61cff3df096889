// Host runtime of libmjp: error reporting, options, model generators,
// Poisson windows and plan construction.  No kernels live here.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace mjp {

static thread_local std::string g_last_error;

mjp_status fail(mjp_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

void clear_error() { g_last_error.clear(); }

mjp_status DevBuf::reserve(size_t want) {
    if (want <= bytes && ptr) return MJP_OK;
    release();
    if (want == 0) return MJP_OK;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        return fail(MJP_E_DEVICE, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    bytes = want;
    return MJP_OK;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// Poisson(k | W) terms around the mode by the ratio recurrence
// p_{k+1} = p_k W / (k+1) (the update of Algorithm 2's P_Poisson), anchored at
// the mode in log space so nothing underflows for large W (Algorithm 2's
// starting value exp(-W) is 0 in FP64 once W > 745).
Window poisson_window(double W, const mjp_opts& o) {
    Window w;
    w.W = W;
    if (!(W > 0.0)) return w;
    const int64_t mode = (int64_t)std::floor(W);
    const int64_t span = (int64_t)std::ceil(40.0 * std::sqrt(W) + 200.0);
    const int64_t lo = std::max<int64_t>(0, mode - span);
    const int64_t hi = mode + span;
    std::vector<double> p((size_t)(hi - lo + 1), 0.0);
    p[(size_t)(mode - lo)] = std::exp(-W + (double)mode * std::log(W) - std::lgamma((double)mode + 1.0));
    for (int64_t k = mode + 1; k <= hi; ++k) p[(size_t)(k - lo)] = p[(size_t)(k - 1 - lo)] * W / (double)k;
    for (int64_t k = mode - 1; k >= lo; --k) p[(size_t)(k - lo)] = p[(size_t)(k + 1 - lo)] * (double)(k + 1) / W;
    // right[i] = sum_{k >= lo+i} p_k (smallest terms first), left[i] = sum_{k < lo+i} p_k
    const size_t m = p.size();
    std::vector<double> right(m + 1, 0.0), left(m + 1, 0.0);
    for (size_t i = m; i-- > 0;) right[i] = right[i + 1] + p[i];
    for (size_t i = 0; i < m; ++i) left[i + 1] = left[i] + p[i];
    auto tail_above = [&](int64_t K) {  // sum_{k > K}
        const int64_t i = K + 1 - lo;
        if (i <= 0) return right[0];
        if (i >= (int64_t)m) return 0.0;
        return right[(size_t)i];
    };
    auto tail_below = [&](int64_t L) {  // sum_{k < L}
        const int64_t i = L - lo;
        if (i <= 0) return 0.0;
        if (i >= (int64_t)m) return left[m];
        return left[(size_t)i];
    };
    if (o.k_rule == MJP_K_PAPER) {
        w.K = (int64_t)std::floor(W + 6.0 * std::sqrt(W)) + 1;
        w.L = 0;
    } else {
        const double eps = o.tol / 4.0;
        int64_t K = hi;
        while (K > 0 && tail_above(K - 1) <= eps) --K;
        int64_t L = std::min(lo, K);  // nothing below the window carries weight
        while (L + 1 <= K && tail_below(L + 1) <= eps) ++L;
        w.K = K;
        w.L = L;
    }
    w.eps_right = tail_above(w.K);
    w.eps_left = tail_below(w.L);
    w.residual = w.eps_left + w.eps_right;
    return w;
}

}  // namespace mjp

using namespace mjp;

extern "C" {

const char* mjp_last_error(void) { return g_last_error.c_str(); }

const char* mjp_version(void) { return "libmjp 0.1 (gfx950)"; }

mjp_status mjp_shutdown(void) {
    clear_error();
    int cur = -1;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    mjp_status s = ll_release_all();
    if (s == MJP_OK) s = items_release_all();
    if (have) (void)hipSetDevice(cur);
    return s;
}

void mjp_opts_default(mjp_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->omega_factor = 1.1;
    o->tol = 1e-9;
    o->k_rule = MJP_K_TOL;
    o->truncation = MJP_CONSERVATIVE;
    o->renorm_every = 32;
    o->lump = 1;
    o->k_cap = 10000000;
    o->variant = MJP_VARIANT_AUTO;
}

}  // extern "C"

namespace mjp {

mjp_status check_opts(const mjp_opts* o) {
    MJP_CHECK(o, MJP_E_INVALID_ARG, "opts is NULL");
    MJP_CHECK(std::isfinite(o->omega_factor) && o->omega_factor > 1.0, MJP_E_INVALID_ARG,
              "omega_factor must be > 1 (got %g)", o->omega_factor);
    MJP_CHECK(std::isfinite(o->tol) && o->tol > 0.0 && o->tol < 1.0, MJP_E_INVALID_ARG,
              "tol must lie in (0, 1) (got %g)", o->tol);
    MJP_CHECK(o->k_rule == MJP_K_TOL || o->k_rule == MJP_K_PAPER, MJP_E_INVALID_ARG, "bad k_rule %d",
              o->k_rule);
    MJP_CHECK(o->truncation == MJP_CONSERVATIVE || o->truncation == MJP_LEAKY, MJP_E_INVALID_ARG,
              "bad truncation %d", o->truncation);
    MJP_CHECK(o->renorm_every >= 0, MJP_E_INVALID_ARG, "renorm_every must be >= 0");
    MJP_CHECK(!(o->renorm_every > 0 && o->truncation == MJP_LEAKY), MJP_E_INVALID_ARG,
              "mass renormalisation is only valid under conservative truncation");
    MJP_CHECK(o->lump == 0 || o->lump == 1, MJP_E_INVALID_ARG, "lump must be 0 or 1");
    MJP_CHECK(o->k_cap >= 1 && o->k_cap <= (int64_t)1 << 30, MJP_E_INVALID_ARG, "k_cap out of range");
    MJP_CHECK(o->variant >= MJP_VARIANT_AUTO && o->variant <= MJP_VARIANT_PERSISTENT_TWOJUMP, MJP_E_INVALID_ARG,
              "bad variant %d", o->variant);
    for (int i = 0; i < 6; ++i) MJP_CHECK(o->reserved[i] == 0, MJP_E_INVALID_ARG, "reserved fields must be 0");
    return MJP_OK;
}

mjp_status check_model(const mjp_model* m) {
    MJP_CHECK(m, MJP_E_INVALID_ARG, "model is NULL");
    int np = 0;
    if (m->model == MJP_MODEL_BD) {
        MJP_CHECK(m->dims[0] >= 1 && m->dims[1] == 1, MJP_E_INVALID_ARG, "BD needs dims = {N >= 1, 1}");
        np = 2;
    } else if (m->model == MJP_MODEL_CASCADE2) {
        MJP_CHECK(m->dims[0] >= 1 && m->dims[1] >= 1, MJP_E_INVALID_ARG, "cascade needs dims >= 1");
        MJP_CHECK((int64_t)m->dims[0] * m->dims[1] <= INT32_MAX / 8, MJP_E_INVALID_ARG, "grid too large");
        np = 4;
    } else if (m->model == MJP_MODEL_TWOSTATE) {
        MJP_CHECK(m->dims[0] >= 1 && m->dims[1] == 1, MJP_E_INVALID_ARG, "two-state model needs dims = {N_R >= 1, 1}");
        MJP_CHECK(2 * (int64_t)m->dims[0] <= INT32_MAX / 8, MJP_E_INVALID_ARG, "grid too large");
        np = 4;
    } else if (m->model == MJP_MODEL_AUTOREG) {
        MJP_CHECK(m->dims[0] >= 1 && m->dims[1] >= 1, MJP_E_INVALID_ARG, "autoregulatory model needs dims >= 1");
        MJP_CHECK(2 * (int64_t)m->dims[0] * m->dims[1] <= INT32_MAX / 8, MJP_E_INVALID_ARG, "grid too large");
        np = 6;
    } else {
        return fail(MJP_E_INVALID_ARG, "unknown model %d", m->model);
    }
    for (int i = 0; i < np; ++i)
        MJP_CHECK(std::isfinite(m->theta[i]) && m->theta[i] >= 0.0, MJP_E_INVALID_ARG,
                  "theta[%d] must be finite and >= 0 (got %g)", i, m->theta[i]);
    return MJP_OK;
}

// Exit rate of every state of a built-in model (the -a_nn of Eq. A_def).
int64_t model_states(const mjp_model* m) {
    switch (m->model) {
        case MJP_MODEL_TWOSTATE: return 2 * (int64_t)m->dims[0];
        case MJP_MODEL_AUTOREG: return 2 * (int64_t)m->dims[0] * m->dims[1];
        default: return (int64_t)m->dims[0] * m->dims[1];
    }
}

// Moves out of state s of a built-in model: target (-1 when it leaves the
// grid) and rate, from the model's reactions.  Returns the number of moves.
//   two-state birth-death (Sec. 3.1.2, Eq. 2S_chem), theta = {beta, gamma,
//     lambda_act, lambda_ina}, s = n_R + g N_R (g = 0 active): active births
//     at beta, deaths at gamma n_R, active -> inactive at lambda_ina,
//     inactive -> active at lambda_act (the text's labels; a birth never
//     crosses into the other gene state);
//   autoregulatory network (Sec. 3.1.3, Eq. STS_chem), theta = {beta_R,
//     beta_P, gamma_R, gamma_P, lambda_act, lambda_ina}, s = n_R + n_P N_R +
//     g N_R N_P: active R births at beta_R, P births at beta_P n_R, deaths at
//     gamma_R n_R and gamma_P n_P, active + P -> inactive at lambda_ina n_P,
//     inactive -> active + P at lambda_act.
struct Move { int64_t to; double rate; };
static int model_moves(const mjp_model* m, int64_t s, Move* mv) {
    int k = 0;
    const double* th = m->theta;
    if (m->model == MJP_MODEL_BD) {
        const int64_t N = m->dims[0];
        mv[k++] = {s + 1 < N ? s + 1 : -1, th[0]};
        if (s >= 1) mv[k++] = {s - 1, th[1] * (double)s};
    } else if (m->model == MJP_MODEL_CASCADE2) {
        const int64_t S1 = m->dims[0], S2 = m->dims[1];
        const int64_t x = s % S1, y = s / S1;
        mv[k++] = {x + 1 < S1 ? s + 1 : -1, th[0]};
        if (x >= 1) mv[k++] = {s - 1, th[1] * (double)x};
        mv[k++] = {y + 1 < S2 ? s + S1 : -1, th[2] * (double)x};
        if (y >= 1) mv[k++] = {s - S1, th[3] * (double)y};
    } else if (m->model == MJP_MODEL_TWOSTATE) {
        const int64_t NR = m->dims[0];
        const int64_t r = s % NR, g = s / NR;
        if (g == 0) mv[k++] = {r + 1 < NR ? s + 1 : -1, th[0]};
        if (r >= 1) mv[k++] = {s - 1, th[1] * (double)r};
        if (g == 0) mv[k++] = {s + NR, th[3]};
        else mv[k++] = {s - NR, th[2]};
    } else {  // MJP_MODEL_AUTOREG
        const int64_t NR = m->dims[0], NP = m->dims[1], plane = NR * NP;
        const int64_t r = s % NR, p = (s / NR) % NP, g = s / plane;
        if (g == 0) mv[k++] = {r + 1 < NR ? s + 1 : -1, th[0]};
        mv[k++] = {p + 1 < NP ? s + NR : -1, th[1] * (double)r};
        if (r >= 1) mv[k++] = {s - 1, th[2] * (double)r};
        if (p >= 1) mv[k++] = {s - NR, th[3] * (double)p};
        if (g == 0 && p >= 1) mv[k++] = {s + plane - NR, th[5] * (double)p};
        if (g == 1) mv[k++] = {p + 1 < NP ? s - plane + NR : -1, th[4]};
    }
    return k;
}

double model_max_exit(const mjp_model* m, int leaky) {
    double best = 0.0;
    if (m->model == MJP_MODEL_TWOSTATE || m->model == MJP_MODEL_AUTOREG) {
        const int64_t n = model_states(m);
        Move mv[8];
        for (int64_t s = 0; s < n; ++s) {
            double e = 0.0;
            const int k = model_moves(m, s, mv);
            for (int i = 0; i < k; ++i)
                if (mv[i].to >= 0 || leaky) e += mv[i].rate;
            best = std::max(best, e);
        }
        return best;
    }
    if (m->model == MJP_MODEL_BD) {
        const int32_t N = m->dims[0];
        const double beta = m->theta[0], gamma = m->theta[1];
        for (int32_t n = 0; n < N; ++n) {
            const double e = ((n + 1 < N || leaky) ? beta : 0.0) + gamma * n;
            best = std::max(best, e);
        }
    } else {
        const int32_t S1 = m->dims[0], S2 = m->dims[1];
        const double k1 = m->theta[0], g1 = m->theta[1], k2 = m->theta[2], g2 = m->theta[3];
        // the exit rate grows with n2, and with n1 except for the dropped
        // boundary birth, so only the last two rows/columns can hold the max
        for (int32_t n2 = std::max(0, S2 - 2); n2 < S2; ++n2)
            for (int32_t n1 = std::max(0, S1 - 2); n1 < S1; ++n1) {
                const double e = ((n1 + 1 < S1 || leaky) ? k1 : 0.0) + g1 * n1 +
                                 ((n2 + 1 < S2 || leaky) ? k2 * n1 : 0.0) + g2 * n2;
                best = std::max(best, e);
            }
    }
    return best;
}

}  // namespace mjp

extern "C" {

mjp_status mjp_model_csr_size(const mjp_model* m, int32_t truncation, int32_t* n_h, int32_t* nnz_h) {
    clear_error();
    mjp_status st = check_model(m);
    if (st) return st;
    MJP_CHECK(n_h && nnz_h, MJP_E_INVALID_ARG, "null output pointer");
    MJP_CHECK(truncation == MJP_CONSERVATIVE || truncation == MJP_LEAKY, MJP_E_INVALID_ARG, "bad truncation");
    int64_t n = 0, nnz = 0;
    if (m->model == MJP_MODEL_BD) {
        const int32_t N = m->dims[0];
        n = N;
        nnz = N;
        if (m->theta[0] != 0.0) nnz += N - 1;          // births n -> n+1
        if (m->theta[1] != 0.0) nnz += N - 1;          // deaths n -> n-1, n >= 1
    } else if (m->model == MJP_MODEL_TWOSTATE || m->model == MJP_MODEL_AUTOREG) {
        n = model_states(m);
        nnz = n;
        Move mv[8];
        for (int64_t s = 0; s < n; ++s) {
            const int k = model_moves(m, s, mv);
            for (int i = 0; i < k; ++i) nnz += (mv[i].to >= 0 && mv[i].rate != 0.0) ? 1 : 0;
        }
    } else {
        const int64_t S1 = m->dims[0], S2 = m->dims[1];
        n = S1 * S2;
        nnz = n;
        if (m->theta[0] != 0.0) nnz += (S1 - 1) * S2;          // k1
        if (m->theta[1] != 0.0) nnz += (S1 - 1) * S2;          // g1 n1, n1 >= 1
        if (m->theta[2] != 0.0) nnz += (S1 - 1) * (S2 - 1);    // k2 n1, n1 >= 1
        if (m->theta[3] != 0.0) nnz += S1 * (S2 - 1);          // g2 n2, n2 >= 1
    }
    MJP_CHECK(nnz <= INT32_MAX, MJP_E_INVALID_ARG, "generator too large for int32 indices");
    *n_h = (int32_t)n;
    *nnz_h = (int32_t)nnz;
    return MJP_OK;
}

mjp_status mjp_model_csr(const mjp_model* m, int32_t truncation, int32_t* row_ptr, int32_t* col_idx,
                         double* val) {
    int32_t n = 0, nnz = 0;
    mjp_status st = mjp_model_csr_size(m, truncation, &n, &nnz);
    if (st) return st;
    MJP_CHECK(row_ptr && col_idx && val, MJP_E_INVALID_ARG, "null output array");
    const int leaky = truncation == MJP_LEAKY;
    int32_t e = 0;
    // one row = one from-state; entries in increasing column order
    struct Ent { int32_t c; double v; };
    if (m->model == MJP_MODEL_TWOSTATE || m->model == MJP_MODEL_AUTOREG) {
        Move mv[8];
        for (int32_t s = 0; s < n; ++s) {
            row_ptr[s] = e;
            Ent ent[9];
            int ne = 0;
            double exit = 0.0;
            const int k = model_moves(m, s, mv);
            for (int i = 0; i < k; ++i) {
                if (mv[i].rate == 0.0) continue;
                if (mv[i].to >= 0) {
                    ent[ne++] = {(int32_t)mv[i].to, mv[i].rate};
                    exit += mv[i].rate;
                } else if (leaky) {
                    exit += mv[i].rate;
                }
            }
            ent[ne++] = {s, -exit};
            std::sort(ent, ent + ne, [](const Ent& a, const Ent& b) { return a.c < b.c; });
            for (int i = 0; i < ne; ++i) { col_idx[e] = ent[i].c; val[e] = ent[i].v; ++e; }
        }
        row_ptr[n] = e;
    } else if (m->model == MJP_MODEL_BD) {
        const int32_t N = m->dims[0];
        const double beta = m->theta[0], gamma = m->theta[1];
        for (int32_t s = 0; s < N; ++s) {
            row_ptr[s] = e;
            const double down = gamma * s;
            const bool up_in = s + 1 < N;
            double exit = down + ((up_in || leaky) ? beta : 0.0);
            if (s > 0 && down != 0.0) { col_idx[e] = s - 1; val[e] = down; ++e; }
            col_idx[e] = s; val[e] = -exit; ++e;
            if (up_in && beta != 0.0) { col_idx[e] = s + 1; val[e] = beta; ++e; }
        }
        row_ptr[N] = e;
    } else {
        const int32_t S1 = m->dims[0], S2 = m->dims[1];
        const double k1 = m->theta[0], g1 = m->theta[1], k2 = m->theta[2], g2 = m->theta[3];
        int32_t s = 0;
        for (int32_t y = 0; y < S2; ++y) {
            for (int32_t x = 0; x < S1; ++x, ++s) {
                row_ptr[s] = e;
                Ent ent[5];
                int ne = 0;
                double exit = 0.0;
                // reactions: (dx, dy, rate)
                const double rate[4] = {k1, g1 * x, k2 * x, g2 * y};
                const int dx[4] = {+1, -1, 0, 0}, dy[4] = {0, 0, +1, -1};
                for (int r = 0; r < 4; ++r) {
                    if (rate[r] == 0.0) continue;
                    const int32_t tx = x + dx[r], ty = y + dy[r];
                    const bool inside = tx >= 0 && tx < S1 && ty >= 0 && ty < S2;
                    if (inside) {
                        ent[ne++] = {tx + S1 * ty, rate[r]};
                        exit += rate[r];
                    } else if (leaky) {
                        exit += rate[r];
                    }
                }
                ent[ne++] = {s, -exit};
                std::sort(ent, ent + ne, [](const Ent& a, const Ent& b) { return a.c < b.c; });
                for (int i = 0; i < ne; ++i) { col_idx[e] = ent[i].c; val[e] = ent[i].v; ++e; }
            }
        }
        row_ptr[s] = e;
    }
    MJP_CHECK(e == nnz, MJP_E_INVALID_ARG, "internal: nnz mismatch %d vs %d", e, nnz);
    return MJP_OK;
}

int32_t mjp_plan_n(const mjp_plan* p) { return p ? p->n : 0; }

void mjp_plan_destroy(mjp_plan* p) {
    if (!p) return;
    int prev = 0;
    bool restore = hipGetDevice(&prev) == hipSuccess;
    if (restore) (void)hipSetDevice(p->device);
    p->slice_off.release();
    p->col.release();
    p->val.release();
    p->dlo.release();
    for (auto& b : p->rho) b.release();
    p->comp.release();
    p->wait.release();
    p->sflag.release();
    p->p2tab.release();
    p->wtab.release();
    p->tinfo.release();
    p->partials.release();
    p->scal.release();
    p->sync.release();
    if (restore) (void)hipSetDevice(prev);
    delete p;
}

}  // extern "C"

namespace mjp {
// Structure, sign and row-sum checks of a generator in CSR form (Eq. A_def:
// non-negative off-diagonal rates, rows summing to 0, or to <= 0 when
// leaky).  Returns m_theta = max |a_nn| and the diagonal.
mjp_status check_generator_csr(const mjp_csr* A, int leaky, double* m_theta_out, std::vector<double>* diag_out) {
    MJP_CHECK(A, MJP_E_INVALID_ARG, "A is NULL");
    const int32_t n = A->n;
    MJP_CHECK(n >= 1, MJP_E_INVALID_ARG, "n must be >= 1 (got %d)", n);
    MJP_CHECK(A->nnz >= 0, MJP_E_INVALID_ARG, "nnz must be >= 0");
    MJP_CHECK(A->row_ptr && (A->nnz == 0 || (A->col_idx && A->val)), MJP_E_INVALID_ARG,
              "null CSR array");
    MJP_CHECK(A->row_ptr[0] == 0 && A->row_ptr[n] == A->nnz, MJP_E_INVALID_ARG,
              "row_ptr must start at 0 and end at nnz");
    double m_theta = 0.0;
    std::vector<double>& diag = *diag_out;
    diag.assign((size_t)n, 0.0);
    for (int32_t r = 0; r < n; ++r) {
        const int32_t b = A->row_ptr[r], e = A->row_ptr[r + 1];
        MJP_CHECK(b <= e, MJP_E_INVALID_ARG, "row_ptr decreases at row %d", r);
        int32_t prev = -1;
        for (int32_t i = b; i < e; ++i) {
            const int32_t c = A->col_idx[i];
            const double v = A->val[i];
            MJP_CHECK(c >= 0 && c < n, MJP_E_INVALID_ARG, "column %d out of range in row %d", c, r);
            MJP_CHECK(c > prev, MJP_E_INVALID_ARG, "columns of row %d not strictly increasing", r);
            MJP_CHECK(std::isfinite(v), MJP_E_INVALID_ARG, "non-finite entry in row %d", r);
            prev = c;
            if (c == r) diag[(size_t)r] = v;
            else MJP_CHECK(v >= 0.0, MJP_E_NOT_GENERATOR, "negative off-diagonal rate in row %d", r);
        }
        m_theta = std::max(m_theta, std::fabs(diag[(size_t)r]));
    }
    for (int32_t r = 0; r < n; ++r) {
        double off = 0.0;
        for (int32_t i = A->row_ptr[r]; i < A->row_ptr[r + 1]; ++i)
            if (A->col_idx[i] != r) off += A->val[i];
        const double rowsum = off + diag[(size_t)r];
        const double slack = 1e-12 * std::max(m_theta, 1e-300);
        if (leaky)
            MJP_CHECK(rowsum <= slack, MJP_E_NOT_GENERATOR,
                      "row %d sums to %g > 0 (a generator row must not gain mass)", r, rowsum);
        else
            MJP_CHECK(std::fabs(rowsum) <= slack, MJP_E_NOT_GENERATOR,
                      "row %d sums to %g, not 0 (conservative truncation)", r, rowsum);
    }
    *m_theta_out = m_theta;
    return MJP_OK;
}
}  // namespace mjp

extern "C" {

mjp_status mjp_plan_create_csr(const mjp_csr* A, const mjp_opts* opts, mjp_plan** out) {
    clear_error();
    MJP_CHECK(out, MJP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    MJP_CHECK(A, MJP_E_INVALID_ARG, "A is NULL");
    mjp_status st = check_opts(opts);
    if (st) return st;
    const int leaky = opts->truncation == MJP_LEAKY;
    double m_theta = 0.0;
    std::vector<double> diag;
    if ((st = check_generator_csr(A, leaky, &m_theta, &diag))) return st;
    const int32_t n = A->n;

    mjp_plan* p = new (std::nothrow) mjp_plan();
    MJP_CHECK(p, MJP_E_DEVICE, "out of host memory");
    p->kind = PLAN_CSR;
    p->n = n;
    p->opts = *opts;
    p->m_theta = m_theta;
    p->omega = opts->omega_factor * m_theta;
    p->nnz = A->nnz;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(MJP_E_DEVICE, "no HIP device available");
    }

    // B = I + A/Omega in FP32, pull form (row m of B^T lists b_nm over n).
    // The diagonal is held as an unevaluated pair of FP32 numbers hi + lo:
    // b_nn = (exact row sum of B) - (FP64 sum of the row's FP32
    // off-diagonals), hi = fl(b_nn), lo = fl(b_nn - hi).  Each row of B then
    // sums to the exact row sum (1 under conservative truncation,
    // 1 - leaked rate/Omega under the leaky reading) to ~1e-16.  A single
    // FP32 diagonal leaves up to 2^-25 per row, a state-dependent gain or
    // loss of mass that the same state repeats at every jump; over thousands
    // of jumps it distorts the result far more than the rounding of the
    // off-diagonal rates, which conserves mass.  Entry 0 of every pull row is
    // the diagonal (column = the row itself); lo is stored per row.
    const double omega = p->omega > 0.0 ? p->omega : 1.0;
    std::vector<int32_t> cnt((size_t)n + 1, 0);
    std::vector<float> bdiag((size_t)n), bdlo((size_t)n);
    for (int32_t r = 0; r < n; ++r) {
        double off = 0.0;
        for (int32_t i = A->row_ptr[r]; i < A->row_ptr[r + 1]; ++i) {
            const int32_t c = A->col_idx[i];
            if (c == r) continue;
            off += (double)(float)(A->val[i] / omega);
            cnt[(size_t)c]++;
        }
        double target = 1.0;
        if (leaky) {
            double exact_off = 0.0;
            for (int32_t i = A->row_ptr[r]; i < A->row_ptr[r + 1]; ++i)
                if (A->col_idx[i] != r) exact_off += A->val[i];
            target = 1.0 + (exact_off + diag[(size_t)r]) / omega;
        }
        const double dex = target - off;
        bdiag[(size_t)r] = (float)dex;
        bdlo[(size_t)r] = (float)(dex - (double)bdiag[(size_t)r]);
        cnt[(size_t)r]++;  // the diagonal is always present in B
    }
    const int32_t n_slices = (n + kSlice - 1) / kSlice;
    std::vector<int32_t> slice_off((size_t)n_slices + 1, 0);
    int32_t max_w = 0;
    for (int32_t s = 0; s < n_slices; ++s) {
        int32_t w = 0;
        for (int32_t r = s * kSlice; r < std::min(n, (s + 1) * kSlice); ++r) w = std::max(w, cnt[(size_t)r]);
        max_w = std::max(max_w, w);
        const int64_t next = (int64_t)slice_off[(size_t)s] + (int64_t)w * kSlice;
        if (next > INT32_MAX) { delete p; return fail(MJP_E_WORKSPACE, "operator too large"); }
        slice_off[(size_t)s + 1] = (int32_t)next;
    }
    const int64_t total = slice_off[(size_t)n_slices];
    std::vector<int32_t> hcol((size_t)total);
    std::vector<float> hval((size_t)total, 0.0f);
    std::vector<int32_t> fill((size_t)n, 0);
    // padding: column = own row, value 0
    for (int32_t s = 0; s < n_slices; ++s) {
        const int32_t w = (slice_off[(size_t)s + 1] - slice_off[(size_t)s]) / kSlice;
        for (int32_t j = 0; j < w; ++j)
            for (int32_t l = 0; l < kSlice; ++l) {
                const int32_t r = std::min(n - 1, s * kSlice + l);
                hcol[(size_t)slice_off[(size_t)s] + (size_t)j * kSlice + l] = r;
            }
    }
    auto put = [&](int32_t m, int32_t src, float v) {
        const int32_t s = m / kSlice, l = m % kSlice;
        const size_t at = (size_t)slice_off[(size_t)s] + (size_t)fill[(size_t)m] * kSlice + l;
        hcol[at] = src;
        hval[at] = v;
        fill[(size_t)m]++;
    };
    for (int32_t r = 0; r < n; ++r) put(r, r, bdiag[(size_t)r]);  // entry 0: the diagonal
    for (int32_t r = 0; r < n; ++r) {  // r = source state n; entries go to output row m = col
        for (int32_t i = A->row_ptr[r]; i < A->row_ptr[r + 1]; ++i) {
            const int32_t c = A->col_idx[i];
            if (c != r) put(c, r, (float)(A->val[i] / omega));
        }
    }
    p->slice_cmin.assign((size_t)n_slices, INT32_MAX);
    p->slice_cmax.assign((size_t)n_slices, -1);
    for (int32_t s = 0; s < n_slices; ++s)
        for (int64_t e = slice_off[(size_t)s]; e < slice_off[(size_t)s + 1]; ++e) {
            p->slice_cmin[(size_t)s] = std::min(p->slice_cmin[(size_t)s], hcol[(size_t)e]);
            p->slice_cmax[(size_t)s] = std::max(p->slice_cmax[(size_t)s], hcol[(size_t)e]);
        }
    p->n_slices = n_slices;
    p->sell_entries = total;
    p->max_width = max_w;
    if ((st = p->slice_off.reserve(sizeof(int32_t) * slice_off.size())) ||
        (st = p->col.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1))) ||
        (st = p->val.reserve(sizeof(float) * (size_t)std::max<int64_t>(total, 1))) ||
        (st = p->dlo.reserve(sizeof(float) * (size_t)std::max<int32_t>(n, 1)))) {
        mjp_plan_destroy(p);
        return st;
    }
    hipError_t e1 = hipMemcpy(p->slice_off.ptr, slice_off.data(), sizeof(int32_t) * slice_off.size(),
                              hipMemcpyHostToDevice);
    hipError_t e2 = total ? hipMemcpy(p->col.ptr, hcol.data(), sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice)
                          : hipSuccess;
    hipError_t e3 = total ? hipMemcpy(p->val.ptr, hval.data(), sizeof(float) * (size_t)total, hipMemcpyHostToDevice)
                          : hipSuccess;
    hipError_t e4 = hipMemcpy(p->dlo.ptr, bdlo.data(), sizeof(float) * (size_t)n, hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
        mjp_plan_destroy(p);
        return fail(MJP_E_DEVICE, "upload of the operator failed");
    }
    *out = p;
    return MJP_OK;
}

mjp_status mjp_plan_create_stencil(const mjp_model* m, const mjp_opts* opts, mjp_plan** out) {
    clear_error();
    MJP_CHECK(out, MJP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mjp_status st = check_model(m);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    mjp_plan* p = new (std::nothrow) mjp_plan();
    MJP_CHECK(p, MJP_E_DEVICE, "out of host memory");
    p->kind = PLAN_STENCIL;
    p->model = *m;
    p->opts = *opts;
    p->n = (int32_t)model_states(m);
    const int leaky = opts->truncation == MJP_LEAKY;
    p->m_theta = model_max_exit(m, leaky);
    p->omega = opts->omega_factor * p->m_theta;
    const double omega = p->omega > 0.0 ? p->omega : 1.0;
    const int np = m->model == MJP_MODEL_BD ? 2 : (m->model == MJP_MODEL_AUTOREG ? 6 : 4);
    for (int i = 0; i < 6; ++i) p->coef.c[i] = i < np ? (float)(m->theta[i] / omega) : 0.0f;
    p->coef.S1 = m->dims[0];
    p->coef.S2 = m->dims[1];
    p->coef.model = m->model;
    p->coef.leaky = leaky;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(MJP_E_DEVICE, "no HIP device available");
    }
    *out = p;
    return MJP_OK;
}

}  // extern "C"
