// Internal declarations shared by the libmjp translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "mjp.h"

namespace mjp {

// ---------------------------------------------------------------- errors
mjp_status fail(mjp_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// A failed HIP call is reported through the library's status and message;
// HIP's per-thread last-error slot is cleared so the caller's next HIP call
// does not report it again.
#define MJP_HIP(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            (void)hipGetLastError();                                                      \
            return ::mjp::fail(MJP_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
        }                                                                                 \
    } while (0)

#define MJP_CHECK(cond, status, ...)                 \
    do {                                             \
        if (!(cond)) return ::mjp::fail(status, __VA_ARGS__); \
    } while (0)

// ------------------------------------------------------ device buffers
// A growable device allocation owned by a plan (or surrogate).
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    mjp_status reserve(size_t want);  // grows (never shrinks); contents not kept
    void release();
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// --------------------------------------------------- Poisson window (FP64)
// Jump window of one collection time: the series keeps k = L..K.
struct Window {
    double t = 0, W = 0;
    double eps_left = 0, eps_right = 0, residual = 0;
    int64_t K = 0, L = 0;
};
// Chooses K and L for W = Omega t under opts (tolerance rule or the paper's
// loop bound); residual = eps_left + eps_right.
Window poisson_window(double W, const mjp_opts& o);

// ------------------------------------------------------------- plans
enum PlanKind { PLAN_CSR = 0, PLAN_STENCIL = 1 };

// FP32 coefficients of a built-in model's B = I + A/Omega, one per reaction
// channel (the diagonal is formed from them in the kernels).
struct StencilCoef {
    float c[6];     // rate / Omega per channel, in the order of the model's theta (mjp.h)
    int32_t S1, S2; // dims: BD {N, 1}; cascade {S1, S2}; two-state {N_R, 1}; autoregulatory {N_R, N_P}
    int32_t model;
    int32_t leaky;
};

constexpr int kSlice = 64;  // rows per sliced-ELL slice (= one wavefront)

// A diagonal entry b_nn of B (FP64 value d) as an unevaluated pair of FP32
// numbers hi + lo with hi = fl(d), lo = fl(d - hi): every FP32 row of B then
// sums to its exact row sum to ~1e-16.  A row is formed as
//   acc = lo x_m;  acc = fma(hi, x_m, acc);  acc = fma(b_nm, x_n, acc) ...
// in every FP32 sweep, so all sweeps give the same bits.
__host__ __device__ __forceinline__ void diag_pair(double d, float& hi, float& lo) {
    hi = (float)d;
    lo = (float)(d - (double)hi);
}


// mjp_loglik with an optional device mask [B] of the items to compute
// (0: skipped, outputs untouched); no host synchronisation (loglik.hip).
mjp_status loglik_run(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d, const mjp_obs* obs,
                      const mjp_opts* opts, const uint8_t* active_d, double* loglik_d, mjp_info* info_d,
                      hipStream_t s);

// Library-owned device state, freed by mjp_shutdown (loglik.hip, expv.hip).
mjp_status ll_release_all();
mjp_status items_release_all();

// Generator checks shared by every CSR entry point (see runtime.hip).
mjp_status check_generator_csr(const mjp_csr* A, int leaky, double* m_theta, std::vector<double>* diag);
// Model description checks (model id, dims, finite non-negative rates).
mjp_status check_model(const mjp_model* m);

}  // namespace mjp

struct mjp_plan {
    int kind = mjp::PLAN_CSR;
    int device = 0;
    int32_t n = 0;
    mjp_opts opts{};
    double m_theta = 0.0;  // max |a_nn|
    double omega = 0.0;    // opts.omega_factor * m_theta

    // CSR plans: B^T in sliced ELL (slice = 64 consecutive output rows,
    // entry j of row r at slice_off[r/64] + 64*j + r%64).
    int32_t n_slices = 0;
    int64_t sell_entries = 0;
    int64_t nnz = 0;
    int32_t max_width = 0;
    std::vector<int32_t> slice_cmin, slice_cmax;  // column span of each slice (host)
    mjp::DevBuf slice_off;  // int32[n_slices+1]
    mjp::DevBuf col;        // int32[sell_entries]
    mjp::DevBuf val;        // float[sell_entries]; entry 0 of each row is the diagonal's hi part
    mjp::DevBuf dlo;        // float[n]: lo part of each row's diagonal (b_nn = hi + lo)

    // stencil plans
    mjp_model model{};
    mjp::StencilCoef coef{};

    // workspace
    mjp::DevBuf rho[2];     // float[N] ping-pong iterate
    mjp::DevBuf comp;       // float[n_t * N] Kahan compensation terms
    mjp::DevBuf wtab;       // double weights, per time k = L..K
    mjp::DevBuf tinfo;      // per-time device parameters
    mjp::DevBuf partials;   // float per-block partial sums
    mjp::DevBuf scal;       // device scalars (masses, scale, flags)
    mjp::DevBuf sync;       // persistent-kernel barrier words, flags, partials
    mjp::DevBuf wait;       // persistent kernel: per-workgroup neighbour interval
    mjp::DevBuf sflag;      // persistent kernel: per-slice local / exported bits
    int wait_key[3] = {0, 0, 0};  // (G, R, valid) the two tables were built for
    mjp::DevBuf p2tab;      // two-jump persistent kernel: per-workgroup regions and neighbour interval
    int p2_key[2] = {0, 0};       // (G, state) the table was built for: 1 fits, 2 does not
    mjp::DevBuf mjtab;      // tiled multi-jump kernel: per-workgroup rings, entry maps, exchange positions
    int mj_key[3] = {0, 0, 0};    // (capacity, W, state) the table was built for: 1 fits, 2 does not
    int mj_G = 0;                 // its workgroups
    int last_path = 0;            // MJP_PATH_* of the last sweep
    std::vector<char> host_stage;
};
