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

// scalar slots in plan->scal (doubles)
enum { S_MASS0 = 0, S_MASSK = 1, S_FLAGS = 2, S_SCALE = 3, S_COUNT = 8 };


struct PersistCfg {
    int R = 0, W = 0, G = 0;
    bool coh = true;  // device-scope iterate accesses (true) or the fenced protocol
    int jumps = 1;    // jumps per synchronisation (2: the two-jump kernel)
    const void* fn = nullptr;
};

bool persistent_fits(const mjp_plan* p, int max_open, bool coh, PersistCfg& cfg);
// the two-jump kernel (device-scope protocol only); builds its tables
bool persistent2_fits(mjp_plan* p, int max_open, PersistCfg& cfg);
mjp_status probe_exchange(mjp_plan* p, int rounds, hipStream_t st, float* ms_out);
mjp_status launch_persistent(mjp_plan* p, const PersistCfg& cfg, const float* rho0, const AllTimes& at,
                             const std::vector<int>& slot, float* out, hipStream_t st);

}  // namespace mjp
