// R-MJP expansion on the GPU: rho(t) = sum_{k=L..K} w_k rho(0) B^k + r rho(0) B^K
// (Algorithm 2 with a left cut L and the residual r lumped onto the last
// iterate), for several collection times in one sweep of jumps.
//
// Kernels:
//   k_weights      FP64 log-space Poisson weights w_k for k in [L, K] per time
//   k_first        k = 0: reads rho(0), checks it, accumulates w_0 rho(0)
//   k_sell_step    one jump rho_k = rho_{k-1} B with B^T in sliced ELL, fused
//                  with the Kahan accumulation of the active times and the
//                  per-block mass partial sums
//   k_stencil_step the same for a built-in model, entries of B computed on
//                  the fly
//   k_accumulate   accumulation only (times beyond the fused capacity)
//   k_reduce       FP64 sum of block partials -> mass, scale, flags
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "internal.h"
#include "sweep.h"

namespace mjp {

mjp_status check_opts(const mjp_opts* o);

constexpr int kBlock = 256;
constexpr int kMaxFused = 6;     // active times accumulated inside a step kernel

struct TimeSet {
    int32_t n;
    TimeParam tp[kMaxFused];
    int32_t slot[kMaxFused];  // compensation-buffer row of each active time
};


// ------------------------------------------------------------- helpers

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Row block of a step kernel.  Workgroups are dispatched round-robin over
// the 8 XCDs; the step launches are padded to a multiple of 8 blocks and
// renumbered so that each XCD owns one band of consecutive row blocks, whose
// gathers (a grid line away) then mostly hit that XCD's own L2.  Logical
// block b covers the rows physical block b covered before, and writes its
// partial to slot b, so every sum keeps its order.
__device__ __forceinline__ int64_t step_block() {
    const unsigned b = blockIdx.x, G = gridDim.x;
    return (G & 7u) ? (int64_t)b : (int64_t)((b & 7u) * (G >> 3) + (b >> 3));
}

// Block-wide sum of v written by thread 0 to out[slot] (slot < nslots).
__device__ __forceinline__ void block_partial_at(float v, float* out, int64_t slot, int64_t nslots) {
    __shared__ float red[kBlock / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0 && slot < nslots) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) s += red[i];
        out[slot] = s;
    }
}

// Block-wide sum of v written by thread 0 to out[blockIdx.x].
__device__ __forceinline__ void block_partial(float v, float* out) {
    __shared__ float red[kBlock / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) s += red[i];
        out[blockIdx.x] = s;
    }
}

// Kahan accumulation of w * y into (s, c) for one time at jump k.
// s lives in the output row, c in the compensation row; the first term
// initialises both, the last writes the compensated total s - c.
__device__ __forceinline__ void kahan_step(const TimeParam& tp, int k, const double* __restrict__ wtab,
                                           float y, float* __restrict__ srow, float* __restrict__ crow,
                                           int row) {
    const float w = (k == tp.K) ? (float)tp.lastw : (float)wtab[tp.woff + (k - tp.L)];
    float s, c;
    if (k == tp.L) {
        s = w * y;
        c = 0.f;
    } else {
        s = srow[row];
        c = crow[row];
        const float yk = fmaf(w, y, -c);
        const float t = s + yk;
        c = (t - s) - yk;
        s = t;
    }
    if (k == tp.K) {
        srow[row] = s - c;
    } else {
        srow[row] = s;
        crow[row] = c;
    }
}

__device__ __forceinline__ void accumulate_all(const TimeSet& ts, int k, const double* __restrict__ wtab,
                                               float y, float* __restrict__ out, float* __restrict__ comp,
                                               int row, int64_t n) {
    for (int i = 0; i < ts.n; ++i)
        kahan_step(ts.tp[i], k, wtab, y, out + (int64_t)ts.tp[i].out * n, comp + (int64_t)ts.slot[i] * n, row);
}

// ------------------------------------------------------------- kernels

// w_k = exp(-W + k log W - lgamma(k+1)) for k in [L, K] of every time.
__global__ void k_weights(AllTimes at, double* __restrict__ wtab) {
    const int j = blockIdx.y;
    if (j >= at.n) return;
    const TimeParam tp = at.tp[j];
    const int cnt = tp.K - tp.L + 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        wtab[tp.woff + i] = poisson_weight(tp.W, tp.L + i);
    }
}

// k = 0: validate rho(0), mass partials, accumulate the k = 0 term.
__global__ __launch_bounds__(kBlock) void k_first(const float* __restrict__ x, int64_t n, TimeSet ts,
                                                  const double* __restrict__ wtab, float* __restrict__ out,
                                                  float* __restrict__ comp, float* __restrict__ partials,
                                                  unsigned* __restrict__ flags) {
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    float v = 0.f;
    if (row < n) {
        v = x[row];
        if (!(v >= 0.f)) {  // negative or NaN
            atomicOr(flags, (v != v) ? (unsigned)MJP_FLAG_NAN : (unsigned)MJP_FLAG_NEG);
        } else if (isinf(v)) {
            atomicOr(flags, (unsigned)MJP_FLAG_NAN);
        }
        accumulate_all(ts, 0, wtab, v, out, comp, (int)row, n);
    }
    block_partial(v, partials);
}

struct SellArgs {
    const int32_t* __restrict__ slice_off;
    const int32_t* __restrict__ col;
    const float* __restrict__ val;
    const float* __restrict__ dlo;   // lo part of each row's diagonal (entry 0 holds hi)
    const float* __restrict__ x;
    float* __restrict__ y;
    const double* __restrict__ scale;  // null -> 1
    int64_t n;
};

template <bool ACC>
__global__ __launch_bounds__(kBlock) void k_sell_step(SellArgs a, int k, TimeSet ts, const double* __restrict__ wtab,
                                                      float* __restrict__ out, float* __restrict__ comp,
                                                      float* __restrict__ partials) {
    const int64_t blk = step_block();
    const int64_t row = blk * kBlock + threadIdx.x;
    float yv = 0.f;
    if (row < a.n) {
        const int32_t s = (int32_t)(row >> 6), l = (int32_t)(row & 63);
        const int32_t beg = a.slice_off[s];
        const int32_t w = (a.slice_off[s + 1] - beg) >> 6;
        const int32_t* cp = a.col + beg + l;
        const float* vp = a.val + beg + l;
        const float xs = a.x[row];
        float acc = a.dlo[row] * xs;
        acc = fmaf(vp[0], xs, acc);  // entry 0: the diagonal, column = row
        for (int32_t j = 1; j < w; ++j) acc = fmaf(vp[j * 64], a.x[cp[j * 64]], acc);
        yv = a.scale ? (float)(*a.scale) * acc : acc;
        a.y[row] = yv;
        if (ACC) accumulate_all(ts, k, wtab, yv, out, comp, (int)row, a.n);
    }
    block_partial_at(yv, partials, blk, (a.n + kBlock - 1) / kBlock);
}

struct StencilArgs {
    StencilCoef cf;
    const float* __restrict__ x;
    float* __restrict__ y;
    const double* __restrict__ scale;
    int64_t n;
};

// y_m = sum_n x_n b_nm for a built-in model.  The off-diagonal b_nm are the
// FP32 products coef * count; the diagonal of a source state is 1 minus the
// FP64 sum of exactly those FP32 numbers, held as an FP32 pair hi + lo, so
// rows of B sum to 1 to ~1e-16.
__device__ __forceinline__ float stencil_row(const StencilCoef& cf, const float* __restrict__ x, int64_t m) {
    int32_t cc[kStencilMaxW];
    float vv[kStencilMaxW], lo;
    stencil_entries<kStencilMaxW>(cf, m, cc, vv, lo);
    const float xs = x[m];
    float y = lo * xs;
    y = fmaf(vv[0], xs, y);
#pragma unroll
    for (int j = 1; j < kStencilMaxW; ++j) y = fmaf(vv[j], x[cc[j]], y);
    return y;
}

template <bool ACC>
__global__ __launch_bounds__(kBlock) void k_stencil_step(StencilArgs a, int k, TimeSet ts,
                                                         const double* __restrict__ wtab, float* __restrict__ out,
                                                         float* __restrict__ comp, float* __restrict__ partials) {
    const int64_t blk = step_block();
    const int64_t row = blk * kBlock + threadIdx.x;
    float yv = 0.f;
    if (row < a.n) {
        const float acc = stencil_row(a.cf, a.x, row);
        yv = a.scale ? (float)(*a.scale) * acc : acc;
        a.y[row] = yv;
        if (ACC) accumulate_all(ts, k, wtab, yv, out, comp, (int)row, a.n);
    }
    block_partial_at(yv, partials, blk, (a.n + kBlock - 1) / kBlock);
}

__global__ __launch_bounds__(kBlock) void k_accumulate(const float* __restrict__ y, int64_t n, int k, TimeSet ts,
                                                       const double* __restrict__ wtab, float* __restrict__ out,
                                                       float* __restrict__ comp) {
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (row < n) accumulate_all(ts, k, wtab, y[row], out, comp, (int)row, n);
}

// One block: FP64 sum of nparts partials in a fixed order.
//   mode 0: mass0 <- sum            (initial mass)
//   mode 1: scale <- mass0 / sum    (renormalisation before the next jump)
//   mode 2: massk <- sum            (report only)
__global__ __launch_bounds__(1024) void k_reduce(const float* __restrict__ partials, int nparts, double* scal, int mode) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 1024) s += (double)partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double tot = red[0];
        if (mode == 0) {
            scal[S_MASS0] = tot;
        } else if (mode == 1) {
            scal[S_MASSK] = tot;
            scal[S_SCALE] = (tot > 0.0 && scal[S_MASS0] > 0.0) ? scal[S_MASS0] / tot : 1.0;
        } else {
            scal[S_MASSK] = tot;
        }
        if (!(tot == tot) || isinf(tot)) {
            unsigned* fl = reinterpret_cast<unsigned*>(scal + S_FLAGS);
            atomicOr(fl, (unsigned)MJP_FLAG_NAN);
        }
    }
}

// Sum of one output row into partials (for the reported masses).
__global__ __launch_bounds__(kBlock) void k_vecsum(const float* __restrict__ v, int64_t n, float* __restrict__ partials) {
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    block_partial(row < n ? v[row] : 0.f, partials);
}

__global__ void k_init_scalars(double* scal) {
    if (threadIdx.x < S_COUNT) scal[threadIdx.x] = (threadIdx.x == S_SCALE) ? 1.0 : 0.0;
}

// ------------------------------------------------------------- driver

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

struct SweepTime {
    double t;
    Window win;
    int32_t out;  // caller's index
};

// Parameters of the times (sorted by t) in at; returns the number of
// Poisson weights of all their windows.
static int64_t build_times(const mjp_plan* p, const std::vector<SweepTime>& times, AllTimes& at) {
    const int nt = (int)times.size();
    at = AllTimes{};
    at.n = nt;
    int64_t wtotal = 0;
    for (int j = 0; j < nt; ++j) {
        const Window& w = times[j].win;
        TimeParam& tp = at.tp[j];
        tp.W = w.W;
        tp.L = (int32_t)w.L;
        tp.K = (int32_t)w.K;
        tp.woff = (int32_t)wtotal;
        tp.out = times[j].out;
        // weight at the last jump: w_K, plus the residual when lumping
        double wK;
        if (w.W > 0.0) wK = std::exp(-w.W + (double)w.K * std::log(w.W) - std::lgamma((double)w.K + 1.0));
        else wK = 1.0;
        tp.lastw = wK + (p->opts.lump ? w.residual : 0.0);
        wtotal += w.K - w.L + 1;
    }
    return wtotal;
}

// Largest number of windows open at the same jump (= compensation rows or
// register slots needed).
static int max_open_windows(const AllTimes& at) {
    int max_open = 0;
    for (int j = 0; j < at.n; ++j) {
        int open = 0;
        for (int i = 0; i < at.n; ++i)
            if (at.tp[i].L <= at.tp[j].L && at.tp[j].L <= at.tp[i].K) ++open;
        max_open = std::max(max_open, open);
    }
    return max_open;
}

// Colours the windows (sorted by start) onto register slots: a slot is
// reused once its previous window has closed.
static std::vector<int> colour_slots(const AllTimes& at) {
    std::vector<int> slot(at.n, -1);
    std::vector<int32_t> busy_until;  // last jump of each slot's current window
    for (int j = 0; j < at.n; ++j) {
        int q = -1;
        for (size_t i = 0; i < busy_until.size(); ++i)
            if (busy_until[i] < at.tp[j].L) { q = (int)i; break; }
        if (q < 0) { q = (int)busy_until.size(); busy_until.push_back(0); }
        busy_until[(size_t)q] = at.tp[j].K;
        slot[(size_t)j] = q;
    }
    return slot;
}

// One sweep over up to kMaxTimes times sorted by t.
static mjp_status run_sweep(mjp_plan* p, const float* rho0, const std::vector<SweepTime>& times, float* out,
                            hipStream_t st, std::vector<double>* out_mass) {
    const int64_t n = p->n;
    const int nt = (int)times.size();
    const unsigned nblk = (unsigned)((n + kBlock - 1) / kBlock);
    const unsigned nblk8 = (nblk + 7u) & ~7u;  // step launches: a multiple of 8 blocks (see step_block)
    AllTimes at;
    const int64_t wtotal = build_times(p, times, at);
    int32_t Kmax = 0;
    for (int j = 0; j < nt; ++j) Kmax = std::max(Kmax, at.tp[j].K);
    const int max_open = max_open_windows(at);
    mjp_status s;
    if ((s = p->rho[0].reserve(sizeof(float) * n)) || (s = p->rho[1].reserve(sizeof(float) * n)) ||
        (s = p->comp.reserve(sizeof(float) * n * (size_t)std::max(max_open, 1))) ||
        (s = p->wtab.reserve(sizeof(double) * (size_t)std::max<int64_t>(wtotal, 1))) ||
        (s = p->partials.reserve(sizeof(float) * nblk)) || (s = p->scal.reserve(sizeof(double) * S_COUNT)))
        return s;
    double* scal = p->scal.as<double>();
    unsigned* flags = reinterpret_cast<unsigned*>(scal + S_FLAGS);
    float* partials = p->partials.as<float>();
    double* wtab = p->wtab.as<double>();
    float* comp = p->comp.as<float>();

    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, st, scal);
    {
        int32_t maxcnt = 0;
        for (int j = 0; j < nt; ++j) maxcnt = std::max(maxcnt, at.tp[j].K - at.tp[j].L + 1);
        const unsigned gx = (unsigned)std::min<int64_t>((maxcnt + 255) / 256, 1024);
        hipLaunchKernelGGL(k_weights, dim3(gx, nt), dim3(256), 0, st, at, wtab);
    }

    PersistCfg cfg;
    const int var = p->opts.variant;
    const bool coh = var != MJP_VARIANT_PERSISTENT_FENCED;
    // eight (else four) jumps per synchronisation on tiles where the operator
    // is a grid, else two on row blocks where its reach allows, else one
    // (MJP_VARIANT_PERSISTENT_TWOJUMP starts at two)
    const bool multi = var == MJP_VARIANT_AUTO || var == MJP_VARIANT_PERSISTENT;
    bool fits = multi && persistent_mj_fits(p, max_open, cfg);
    if (!fits && (multi || var == MJP_VARIANT_PERSISTENT_TWOJUMP)) fits = persistent2_fits(p, max_open, cfg);
    if (!fits && var != MJP_VARIANT_STEPWISE) fits = persistent_fits(p, max_open, coh, cfg);
    if (fits) {
        const std::vector<int> slot = colour_slots(at);
        p->last_path = cfg.jumps >= 4 ? MJP_PATH_PERSISTENT_MULTIJUMP
                       : cfg.jumps == 2         ? MJP_PATH_PERSISTENT_TWOJUMP
                                                : (coh ? MJP_PATH_PERSISTENT : MJP_PATH_PERSISTENT_FENCED);
        if ((s = launch_persistent(p, cfg, rho0, at, slot, out, st))) return s;
    } else {
        if (var == MJP_VARIANT_PERSISTENT || var == MJP_VARIANT_PERSISTENT_FENCED || var == MJP_VARIANT_PERSISTENT_ONEJUMP ||
            var == MJP_VARIANT_PERSISTENT_TWOJUMP)
            return fail(MJP_E_UNSUPPORTED, "the persistent kernel cannot hold this operator (width %d, %d open windows)",
                        p->max_width, max_open);
        p->last_path = MJP_PATH_STEPWISE;
        // compensation rows are handed out to times while their window is open
        std::vector<int> slot_of(nt, -1);
        std::vector<int> free_slots;
        for (int i = max_open - 1; i >= 0; --i) free_slots.push_back(i);

        auto active_at = [&](int k, std::vector<int>& act) {
            act.clear();
            for (int j = 0; j < nt; ++j)
                if (at.tp[j].L <= k && k <= at.tp[j].K) act.push_back(j);
        };
        std::vector<int> act;
        // Launch the accumulations of jump k for the active times: the first
        // kMaxFused inside the step kernel (through ts), the rest separately.
        auto make_sets = [&](int k, TimeSet& fused, std::vector<TimeSet>& extra) -> mjp_status {
            active_at(k, act);
            fused.n = 0;
            extra.clear();
            for (int j : act) {
                if (slot_of[j] < 0) {
                    if (free_slots.empty()) return fail(MJP_E_WORKSPACE, "internal: compensation rows exhausted");
                    slot_of[j] = free_slots.back();
                    free_slots.pop_back();
                }
                TimeSet* dst = &fused;
                if (fused.n == kMaxFused) {
                    if (extra.empty() || extra.back().n == kMaxFused) extra.push_back(TimeSet{});
                    dst = &extra.back();
                }
                dst->tp[dst->n] = at.tp[j];
                dst->slot[dst->n] = slot_of[j];
                dst->n++;
            }
            return MJP_OK;
        };
        auto release_done = [&](int k) {
            for (int j : act)
                if (at.tp[j].K == k) {
                    free_slots.push_back(slot_of[j]);
                    slot_of[j] = -2;
                }
        };

        TimeSet fused{};
        std::vector<TimeSet> extra;
        if ((s = make_sets(0, fused, extra))) return s;
        hipLaunchKernelGGL(k_first, dim3(nblk), dim3(kBlock), 0, st, rho0, n, fused, wtab, out, comp, partials, flags);
        for (const TimeSet& e : extra)
            hipLaunchKernelGGL(k_accumulate, dim3(nblk), dim3(kBlock), 0, st, rho0, n, 0, e, wtab, out, comp);
        release_done(0);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partials, (int)nblk, scal, 0);

        const int m = p->opts.renorm_every;
        const float* x = rho0;
        for (int k = 1; k <= Kmax; ++k) {
            float* y = p->rho[k & 1].as<float>();
            if ((s = make_sets(k, fused, extra))) return s;
            const double* scale = (m > 0 && (k - 1) > 0 && (k - 1) % m == 0) ? scal + S_SCALE : nullptr;
            if (p->kind == PLAN_CSR) {
                SellArgs a{p->slice_off.as<int32_t>(), p->col.as<int32_t>(), p->val.as<float>(), p->dlo.as<float>(), x, y,
                           scale, n};
                if (fused.n)
                    hipLaunchKernelGGL(k_sell_step<true>, dim3(nblk8), dim3(kBlock), 0, st, a, k, fused, wtab, out, comp, partials);
                else
                    hipLaunchKernelGGL(k_sell_step<false>, dim3(nblk8), dim3(kBlock), 0, st, a, k, fused, wtab, out, comp, partials);
            } else {
                StencilArgs a{p->coef, x, y, scale, n};
                if (fused.n)
                    hipLaunchKernelGGL(k_stencil_step<true>, dim3(nblk8), dim3(kBlock), 0, st, a, k, fused, wtab, out, comp, partials);
                else
                    hipLaunchKernelGGL(k_stencil_step<false>, dim3(nblk8), dim3(kBlock), 0, st, a, k, fused, wtab, out, comp, partials);
            }
            for (const TimeSet& e : extra)
                hipLaunchKernelGGL(k_accumulate, dim3(nblk), dim3(kBlock), 0, st, y, n, k, e, wtab, out, comp);
            release_done(k);
            if (m > 0 && k % m == 0 && k < Kmax)
                hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partials, (int)nblk, scal, 1);
            x = y;
        }
    }
    MJP_HIP(hipGetLastError());
    if (out_mass) {
        out_mass->assign(nt + 1, 0.0);
        // mass of rho(0) and of every output row
        std::vector<double> h(S_COUNT);
        MJP_HIP(hipMemcpyAsync(h.data(), scal, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, st));
        MJP_HIP(hipStreamSynchronize(st));
        (*out_mass)[nt] = h[S_MASS0];
        unsigned fl = 0;
        std::memcpy(&fl, &h[S_FLAGS], sizeof fl);
        for (int j = 0; j < nt; ++j) {
            hipLaunchKernelGGL(k_vecsum, dim3(nblk), dim3(kBlock), 0, st, out + (int64_t)at.tp[j].out * n, n, partials);
            hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partials, (int)nblk, scal, 2);
            MJP_HIP(hipMemcpyAsync(h.data(), scal, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, st));
            MJP_HIP(hipStreamSynchronize(st));
            (*out_mass)[j] = h[S_MASSK];
            unsigned f2 = 0;
            std::memcpy(&f2, &h[S_FLAGS], sizeof f2);
            fl |= f2;
        }
        out_mass->push_back((double)fl);
    }
    return MJP_OK;
}

// Windows already formed in one call, keyed by (W, tol, k_rule): a batch
// of items on one operator and one set of times forms each window once.
struct WindowCache {
    std::map<std::tuple<double, double, int32_t>, Window> m;
    const Window& get(double W, const mjp_opts& o) {
        const auto key = std::make_tuple(W, o.tol, (int32_t)o.k_rule);
        auto it = m.find(key);
        if (it == m.end()) it = m.emplace(key, poisson_window(W, o)).first;
        return it->second;
    }
};

// The times' windows (checked against k_cap), sorted by t; out = caller's index.
static mjp_status prepare_times(const mjp_plan* p, int32_t n_t, const double* t_h, std::vector<SweepTime>& all,
                                WindowCache* cache = nullptr) {
    all.clear();
    all.reserve(n_t);
    for (int32_t j = 0; j < n_t; ++j) {
        const double t = t_h[j];
        MJP_CHECK(std::isfinite(t) && t >= 0.0, MJP_E_INVALID_ARG, "t[%d] = %g must be finite and >= 0", j, t);
        SweepTime s;
        s.t = t;
        s.out = j;
        // W = 0 gives K = L = 0
        s.win = cache ? cache->get(p->omega * t, p->opts) : poisson_window(p->omega * t, p->opts);
        MJP_CHECK(s.win.K <= p->opts.k_cap, MJP_E_K_LIMIT, "t[%d] needs K = %lld > k_cap = %lld", j,
                  (long long)s.win.K, (long long)p->opts.k_cap);
        MJP_CHECK(s.win.K < INT32_MAX / 2, MJP_E_K_LIMIT, "K too large");
        all.push_back(s);
    }
    std::stable_sort(all.begin(), all.end(), [](const SweepTime& a, const SweepTime& b) { return a.t < b.t; });
    return MJP_OK;
}

// Workspaces of the batched sweep per (device, stream), most recently used
// first; the least recently used is freed beyond kItemStreams streams.
constexpr int kItemDevices = 64;
constexpr int kItemStreams = 16;
struct ItemCtx {
    std::mutex mu;
    std::vector<std::unique_ptr<ItemWork>> work;
};

static ItemCtx& item_ctx(int dev) {
    static ItemCtx ctxs[kItemDevices];
    return ctxs[dev];
}

// Frees every batched-sweep workspace on every device.
mjp_status items_release_all() {
    for (int dev = 0; dev < kItemDevices; ++dev) {
        ItemCtx& C = item_ctx(dev);
        std::lock_guard<std::mutex> lock(C.mu);
        if (C.work.empty()) continue;
        MJP_HIP(hipSetDevice(dev));
        MJP_HIP(hipDeviceSynchronize());
        for (auto& w : C.work) w->release();
        C.work.clear();
    }
    return MJP_OK;
}

static mjp_status item_work(ItemCtx& C, hipStream_t st, ItemWork*& out) {
    for (size_t i = 0; i < C.work.size(); ++i)
        if (C.work[i]->stream == st) {
            if (i > 0) std::rotate(C.work.begin(), C.work.begin() + i, C.work.begin() + i + 1);
            out = C.work[0].get();
            return MJP_OK;
        }
    if ((int)C.work.size() >= kItemStreams) {
        MJP_HIP(hipDeviceSynchronize());
        C.work.back()->release();
        C.work.pop_back();
    }
    std::unique_ptr<ItemWork> w(new (std::nothrow) ItemWork());
    MJP_CHECK(w, MJP_E_DEVICE, "out of host memory");
    w->stream = st;
    C.work.insert(C.work.begin(), std::move(w));
    out = C.work[0].get();
    return MJP_OK;
}

}  // namespace mjp

using namespace mjp;

extern "C" mjp_status mjp_expv(mjp_plan* p, const float* rho0_d, int32_t n_t, const double* t_h, float* out_d,
                               mjp_info* info_h, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(p, MJP_E_INVALID_ARG, "plan is NULL");
    MJP_CHECK(rho0_d && out_d && t_h, MJP_E_INVALID_ARG, "null buffer");
    MJP_CHECK(n_t >= 1, MJP_E_INVALID_ARG, "n_t must be >= 1");
    const int64_t n = p->n;
    {
        const char* a = reinterpret_cast<const char*>(rho0_d);
        const char* b = reinterpret_cast<const char*>(out_d);
        MJP_CHECK(a + sizeof(float) * n <= b || b + sizeof(float) * n * n_t <= a, MJP_E_INVALID_ARG,
                  "out_d overlaps rho0_d");
    }
    std::vector<SweepTime> all;
    if (mjp_status s = prepare_times(p, n_t, t_h, all)) return s;
    DeviceGuard g(p->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    std::vector<double> mass;
    for (size_t b = 0; b < all.size(); b += kMaxTimes) {
        std::vector<SweepTime> chunk(all.begin() + b, all.begin() + std::min(all.size(), b + kMaxTimes));
        mjp_status s = run_sweep(p, rho0_d, chunk, out_d, st, info_h ? &mass : nullptr);
        if (s) return s;
        if (info_h) {
            const int nt = (int)chunk.size();
            unsigned flags = (unsigned)mass[nt + 1];
            for (int j = 0; j < nt; ++j) {
                mjp_info& inf = info_h[chunk[j].out];
                std::memset(&inf, 0, sizeof inf);
                inf.omega = p->omega;
                inf.W = chunk[j].win.W;
                inf.eps_left = chunk[j].win.eps_left;
                inf.eps_right = chunk[j].win.eps_right;
                inf.residual = chunk[j].win.residual;
                inf.mass_in = mass[nt];
                inf.mass_out = mass[j];
                inf.K = (int32_t)chunk[j].win.K;
                inf.L = (int32_t)chunk[j].win.L;
                inf.flags = (int32_t)(flags & ~kFlagBarrierTimeout);
                inf.path = p->last_path;
            }
            if (flags & kFlagBarrierTimeout)
                return fail(MJP_E_DEVICE, "a grid barrier of the persistent kernel timed out");
            if (flags & (MJP_FLAG_NAN | MJP_FLAG_NEG))
                return fail(MJP_E_NUMERIC, "numeric flags 0x%x (NaN/Inf or negative entry)", flags);
        }
    }
    return MJP_OK;
}

extern "C" mjp_status mjp_probe_exchange(mjp_plan* p, int32_t rounds, double* us_per_round_h, mjp_stream_t stream) {
    int32_t jumps = 0;
    return mjp_probe_exchange2(p, rounds, us_per_round_h, &jumps, stream);
}

extern "C" mjp_status mjp_probe_exchange2(mjp_plan* p, int32_t rounds, double* us_per_round_h, int32_t* jumps_h,
                                          mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(p && us_per_round_h && jumps_h, MJP_E_INVALID_ARG, "null argument");
    MJP_CHECK(rounds >= 1 && rounds <= 1000000, MJP_E_INVALID_ARG, "rounds must be in [1, 10^6]");
    DeviceGuard guard(p->device);
    float ms = 0.f;
    int jumps = 0;
    const mjp_status s = probe_exchange(p, rounds, reinterpret_cast<hipStream_t>(stream), &ms, &jumps);
    if (s) return s;
    *us_per_round_h = 1e3 * (double)ms / rounds;
    *jumps_h = jumps;
    return MJP_OK;
}

extern "C" mjp_status mjp_expv_batched(int32_t B, mjp_plan* const* plans, const float* const* rho0_d,
                                       const int32_t* n_t, const double* const* t_h, float* const* out_d,
                                       mjp_info* info_h, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(B >= 0, MJP_E_INVALID_ARG, "B must be >= 0");
    if (B == 0) return MJP_OK;
    MJP_CHECK(plans && rho0_d && n_t && t_h && out_d, MJP_E_INVALID_ARG, "null array");
    std::vector<int64_t> ioff((size_t)B + 1, 0);  // first mjp_info entry of each item
    for (int32_t b = 0; b < B; ++b) {
        MJP_CHECK(plans[b] && rho0_d[b] && out_d[b] && t_h[b] && n_t[b] >= 1, MJP_E_INVALID_ARG,
                  "item %d: null or empty argument", b);
        for (int32_t j = 0; j < n_t[b]; ++j)
            MJP_CHECK(std::isfinite(t_h[b][j]) && t_h[b][j] >= 0.0, MJP_E_INVALID_ARG, "item %d: bad time", b);
        const int64_t n = plans[b]->n;
        const char* x = reinterpret_cast<const char*>(rho0_d[b]);
        const char* y = reinterpret_cast<const char*>(out_d[b]);
        MJP_CHECK(x + sizeof(float) * n <= y || y + sizeof(float) * n * n_t[b] <= x, MJP_E_INVALID_ARG,
                  "item %d: out_d overlaps rho0_d", b);
        ioff[(size_t)b + 1] = ioff[(size_t)b] + n_t[b];
    }
    // Items that one workgroup holds (on the first item's device, with the
    // device-scope persistent sweep allowed) go through the batched sweep;
    // the others through their own sweep, one after another.
    const int dev = plans[0]->device;
    std::vector<ItemSweep> items;
    std::vector<int32_t> item_of, single;
    items.reserve((size_t)B);
    item_of.reserve((size_t)B);
    std::vector<std::vector<SweepTime>> times((size_t)B);
    WindowCache wcache;
    for (int32_t b = 0; b < B; ++b) {
        const mjp_plan* p = plans[b];
        if (mjp_status s = prepare_times(p, n_t[b], t_h[b], times[(size_t)b], &wcache)) return s;
        const int var = p->opts.variant;
        bool ok = p->device == dev && n_t[b] <= kMaxTimes &&
                  (var == MJP_VARIANT_AUTO || var == MJP_VARIANT_PERSISTENT || var == MJP_VARIANT_PERSISTENT_ONEJUMP);
        if (ok) {
            ItemSweep it;
            it.p = p;
            it.rho0 = rho0_d[b];
            it.out = out_d[b];
            it.wtotal = build_times(p, times[(size_t)b], it.at);
            ok = item_fits(p, max_open_windows(it.at), it.R, it.W);
            if (ok) {
                const std::vector<int> slot = colour_slots(it.at);
                for (int j = 0; j < it.at.n; ++j) it.slot[j] = slot[(size_t)j];
                items.push_back(it);
                item_of.push_back(b);
            }
        }
        if (!ok) single.push_back(b);
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!items.empty()) {
        MJP_CHECK(dev >= 0 && dev < kItemDevices, MJP_E_UNSUPPORTED, "device %d beyond the supported count", dev);
        DeviceGuard g(dev);
        ItemCtx& C = item_ctx(dev);
        std::lock_guard<std::mutex> lock(C.mu);
        ItemWork* ws = nullptr;
        std::vector<int64_t> roff;
        mjp_status s;
        if ((s = item_work(C, st, ws)) || (s = launch_items(items, info_h != nullptr, *ws, st, roff))) return s;
        if (info_h) {
            const size_t bytes = ws->info.bytes;
            std::vector<double> rep(bytes / sizeof(double));
            MJP_HIP(hipMemcpyAsync(rep.data(), ws->info.ptr, bytes, hipMemcpyDeviceToHost, st));
            MJP_HIP(hipStreamSynchronize(st));
            unsigned bad = 0;
            for (size_t i = 0; i < items.size(); ++i) {
                const int32_t b = item_of[i];
                const mjp_plan* p = plans[b];
                const double* r = rep.data() + roff[i];
                unsigned fl = 0;
                std::memcpy(&fl, r, sizeof fl);
                bad |= fl;
                for (const SweepTime& tt : times[(size_t)b]) {
                    mjp_info& inf = info_h[ioff[(size_t)b] + tt.out];
                    std::memset(&inf, 0, sizeof inf);
                    inf.omega = p->omega;
                    inf.W = tt.win.W;
                    inf.eps_left = tt.win.eps_left;
                    inf.eps_right = tt.win.eps_right;
                    inf.residual = tt.win.residual;
                    inf.mass_in = r[1];
                    inf.mass_out = r[6 + tt.out];
                    inf.K = (int32_t)tt.win.K;
                    inf.L = (int32_t)tt.win.L;
                    inf.flags = (int32_t)fl;
                    inf.path = MJP_PATH_BATCHED_ITEM;
                }
            }
            if (bad & (MJP_FLAG_NAN | MJP_FLAG_NEG))
                return fail(MJP_E_NUMERIC, "numeric flags 0x%x (NaN/Inf or negative entry)", bad);
        }
    }
    for (int32_t b : single) {
        mjp_status s = mjp_expv(plans[b], rho0_d[b], n_t[b], t_h[b], out_d[b],
                                info_h ? info_h + ioff[(size_t)b] : nullptr, stream);
        if (s) return s;
    }
    return MJP_OK;
}
