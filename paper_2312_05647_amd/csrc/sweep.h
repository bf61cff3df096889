// Definitions shared by the stepwise and the persistent sweeps.
#pragma once

#include <vector>

#include "gridsync.h"
#include "internal.h"

namespace mjp {

constexpr int kMaxTimes = 48;  // collection times handled by one sweep

// Per collection time, passed to kernels by value.
struct TimeParam {
    double W;       // Omega t
    double lastw;   // weight applied at k == K: w_K (+ residual when lumping)
    int32_t L, K;   // accumulated window
    int32_t woff;   // offset of w_L in the weight table
    int32_t out;    // row of the output array
};

struct AllTimes {
    int32_t n;
    TimeParam tp[kMaxTimes];
};

// Poisson weight w_k = exp(-W + k log W - lgamma(k + 1)) in log space
// (Algorithm 2's P(k | Omega t)); W = 0 is the point mass at k = 0.
__device__ __forceinline__ double poisson_weight(double W, int k) {
    if (W > 0.0) return exp(-W + (double)k * log(W) - lgamma((double)k + 1.0));
    return k == 0 ? 1.0 : 0.0;
}

// scalar slots in plan->scal (doubles)
enum { S_MASS0 = 0, S_MASSK = 1, S_FLAGS = 2, S_SCALE = 3, S_COUNT = 8 };


// Pull row m of B = I + A/Omega for a built-in model: entries (column,
// value), entry 0 the diagonal's hi part (column m) with its lo part in lo,
// then the inflows in a fixed order per model; unused entries are (m, 0).
// Each inflow value is the FP32 product (rate/Omega) * count that the source
// state's exit uses, and the diagonal is 1 minus the FP64 sum of the row's
// FP32 exits, so rows of B sum to their exact sum to ~1e-16.  Inflows, in
// the moves of the models' generators (Eq. A_def with the rates of Eqs.
// BD_def, Gene_def, autoReg_def and the cascade):
//   BD           m-1 birth beta; m+1 death gamma (n+1)
//   cascade      m-1 birth k1; m+1 death g1 (n1+1); m-S1 birth k2 n1;
//                m+S1 death g2 (n2+1)
//   two-state    m-1 birth beta (active); m+1 death gamma (n_R+1); the other
//                gene state: lambda_act into active, lambda_ina into inactive
//   autoreg      m-1 R birth beta_R (active); m+1 R death gamma_R (n_R+1);
//                m-N_R P birth beta_P n_R; m+N_R P death gamma_P (n_P+1);
//                into inactive (n_R, n_P) binding from active (n_R, n_P+1)
//                at lambda_ina (n_P+1); into active (n_R, n_P) unbinding
//                from inactive (n_R, n_P-1) at lambda_act.
// Births that would leave the grid are dropped (or, leaky, still leave).
constexpr int kStencilMaxW = 6;
__host__ __device__ inline int stencil_width(int model) {
    return model == MJP_MODEL_AUTOREG ? 6 : (model == MJP_MODEL_TWOSTATE ? 4 : (model == MJP_MODEL_BD ? 3 : 5));
}
// farthest column a row reads
__host__ __device__ inline int64_t stencil_reach(const StencilCoef& cf) {
    if (cf.model == MJP_MODEL_BD) return 1;
    if (cf.model == MJP_MODEL_AUTOREG) {
        const int64_t plane = (int64_t)cf.S1 * cf.S2;
        return plane - cf.S1 > cf.S1 ? plane - cf.S1 : cf.S1;
    }
    return cf.S1;
}
template <int W>
__host__ __device__ __forceinline__ void stencil_entries(const StencilCoef& cf, int64_t m, int32_t (&cc)[W], float (&vv)[W],
                                                float& lo) {
    static_assert(W >= 3, "entries");
    const int32_t mi = (int32_t)m;
    float v[kStencilMaxW] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int32_t c[kStencilMaxW] = {mi, mi, mi, mi, mi, mi};
    double exits = 0.0;
    const bool lk = cf.leaky != 0;
    if (cf.model == MJP_MODEL_BD || cf.model == MJP_MODEL_CASCADE2) {
        const int32_t S1 = cf.S1, S2 = cf.model == MJP_MODEL_BD ? 1 : cf.S2;
        const int32_t i2 = cf.model == MJP_MODEL_BD ? 0 : mi / S1, i1 = mi - i2 * S1;
        const float f1 = (float)i1, f2 = (float)i2;
        const float b1 = cf.c[0], d1 = cf.c[1];
        const float b2 = cf.model == MJP_MODEL_BD ? 0.f : cf.c[2], d2 = cf.model == MJP_MODEL_BD ? 0.f : cf.c[3];
        const float o_b1 = (i1 + 1 < S1 || lk) ? b1 : 0.f;
        const float o_d1 = d1 * f1;
        const float o_b2 = (i2 + 1 < S2 || lk) ? b2 * f1 : 0.f;
        const float o_d2 = d2 * f2;
        exits = ((double)o_b1 + (double)o_d1) + ((double)o_b2 + (double)o_d2);
        if (i1 > 0) { c[1] = mi - 1; v[1] = b1; }
        if (i1 + 1 < S1) { c[2] = mi + 1; v[2] = d1 * (f1 + 1.f); }
        if (i2 > 0) { c[3] = mi - S1; v[3] = b2 * f1; }
        if (i2 + 1 < S2) { c[4] = mi + S1; v[4] = d2 * (f2 + 1.f); }
    } else if (cf.model == MJP_MODEL_TWOSTATE) {
        const int32_t NR = cf.S1;
        const bool act = mi < NR;
        const int32_t r = act ? mi : mi - NR;
        const float fr = (float)r;
        const float be = cf.c[0], ga = cf.c[1], la = cf.c[2], li = cf.c[3];
        const float o_b = (act && (r + 1 < NR || lk)) ? be : 0.f;
        const float o_d = ga * fr;
        const float o_s = act ? li : la;
        exits = ((double)o_b + (double)o_d) + (double)o_s;
        if (act && r > 0) { c[1] = mi - 1; v[1] = be; }
        if (r + 1 < NR) { c[2] = mi + 1; v[2] = ga * (fr + 1.f); }
        if (act) { c[3] = mi + NR; v[3] = la; }
        else { c[3] = mi - NR; v[3] = li; }
    } else {  // MJP_MODEL_AUTOREG
        const int32_t NR = cf.S1, NP = cf.S2, plane = NR * NP;
        const bool act = mi < plane;
        const int32_t q = act ? mi : mi - plane;
        const int32_t p = q / NR, r = q - p * NR;
        const float fr = (float)r, fp = (float)p;
        const float bR = cf.c[0], bP = cf.c[1], gR = cf.c[2], gP = cf.c[3], la = cf.c[4], li = cf.c[5];
        const float o_bR = (act && (r + 1 < NR || lk)) ? bR : 0.f;
        const float o_bP = (p + 1 < NP || lk) ? bP * fr : 0.f;
        const float o_dR = gR * fr;
        const float o_dP = gP * fp;
        const float o_sw = act ? li * fp : ((p + 1 < NP || lk) ? la : 0.f);
        exits = (((double)o_bR + (double)o_bP) + ((double)o_dR + (double)o_dP)) + (double)o_sw;
        if (act && r > 0) { c[1] = mi - 1; v[1] = bR; }
        if (r + 1 < NR) { c[2] = mi + 1; v[2] = gR * (fr + 1.f); }
        if (p > 0) { c[3] = mi - NR; v[3] = bP * fr; }
        if (p + 1 < NP) { c[4] = mi + NR; v[4] = gP * (fp + 1.f); }
        if (!act && p + 1 < NP) { c[5] = mi - plane + NR; v[5] = li * (fp + 1.f); }
        if (act && p > 0) { c[5] = mi + plane - NR; v[5] = la; }
    }
    float hi;
    diag_pair(1.0 - exits, hi, lo);
    c[0] = mi;
    v[0] = hi;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        cc[j] = j < kStencilMaxW ? c[j] : mi;
        vv[j] = j < kStencilMaxW ? v[j] : 0.f;
    }
}

struct PersistCfg {
    int R = 0, W = 0, G = 0;
    bool coh = true;  // device-scope iterate accesses (true) or the fenced protocol
    int jumps = 1;    // jumps per synchronisation (2: the two-jump kernel)
    const void* fn = nullptr;
};

bool persistent_fits(const mjp_plan* p, int max_open, bool coh, PersistCfg& cfg);

// ---- batched sweep of operators that one workgroup holds
// One item: an operator, an initial vector and up to kMaxTimes collection
// times, run by one workgroup with the whole vector in LDS (the
// single-workgroup form of the persistent sweep, so its result equals the
// item's own sweep bit for bit).
struct ItemSweep {
    const mjp_plan* p = nullptr;
    const float* rho0 = nullptr;
    float* out = nullptr;
    AllTimes at{};
    int32_t slot[kMaxTimes] = {};
    int R = 0, W = 0;     // rows per thread and entries per row of the kernel that runs it
    int64_t wtotal = 0;   // Poisson weights of all its windows
};
// Workspace of the batched sweep, one per (device, stream).
struct ItemWork {
    hipStream_t stream = nullptr;
    DevBuf args, wtab, info;
    void* stage = nullptr;        // pinned host copy of the argument block
    size_t stage_bytes = 0;
    hipEvent_t staged = nullptr;  // recorded after the last upload from stage
    void release();
};
// Kernel shape (R, W) for an item of plan p with max_open windows open at
// once; false if one workgroup cannot hold it.
bool item_fits(const mjp_plan* p, int max_open, int& R, int& W);
// Launches every item on st: one weights pass, then one launch per kernel
// shape present (items of one operator class: one launch).  info_off[i]:
// offset in doubles of item i's report in ws.info: [0] flags word,
// [1] initial mass, [2] last measured mass, [6 + j] FP64 mass of output row
// j (written only when out_mass).
mjp_status launch_items(const std::vector<ItemSweep>& items, bool out_mass, ItemWork& ws, hipStream_t st,
                        std::vector<int64_t>& info_off);
// the two-jump kernel (device-scope protocol only); builds its tables
bool persistent2_fits(mjp_plan* p, int max_open, PersistCfg& cfg);
// the tiled kernel with eight (else four) jumps per synchronisation
// (grid-structured operators of width <= 5); builds and caches its tables
bool persistent_mj_fits(mjp_plan* p, int max_open, PersistCfg& cfg);
// times `rounds` exchange-only rounds of the plan's two-jump or tiled sweep;
// *jumps_out: the jumps per synchronisation of that sweep
mjp_status probe_exchange(mjp_plan* p, int rounds, hipStream_t st, float* ms_out, int* jumps_out);
mjp_status launch_persistent(mjp_plan* p, const PersistCfg& cfg, const float* rho0, const AllTimes& at,
                             const std::vector<int>& slot, float* out, hipStream_t st);

}  // namespace mjp
