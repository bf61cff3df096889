// Fourth-order Runge-Kutta propagator (Method #4, Sec. 2.2.4, Eqs. RKstep
// and RKintermediate) on the GPU, in FP64, with time-dependent rates.
//
// A(t) = sum_c g_c(t) A_c: every channel A_c is a generator (checked like a
// CSR plan's operator) and g_c(t) >= 0 is piecewise linear through knots set
// by the caller (constant 1 by default), so A(t) is a generator at all t.
// One step of length h from x:
//   k1 = x A(t), k2 = (x + h/2 k1) A(t + h/2), k3 = (x + h/2 k2) A(t + h/2),
//   k4 = (x + h k3) A(t + h),   x <- x + h/6 (k1 + 2 k2 + 2 k3 + k4)
// (the paper's d_i are h k_i).  h = dt_factor / m with m the largest exit
// rate over the schedule (dt_factor 1 is the paper's stability bound); the
// last step before each requested time is shortened to land on it.
//
// Layout: all channels' entries merged into one A^T in sliced ELL (64-row
// slices, column-major inside a slice), FP64 value, int32 source column and
// a one-byte channel per entry.  A stage is one streaming kernel: it gathers
// the stage input, forms k with the stage's g_c (kernel arguments, staged
// in LDS), writes the next stage's input and updates the weighted sum; the
// fourth writes the new x.  Five N-vectors: x (two buffers), two stage
// inputs, the weighted sum.
//
// Stencil form (the birth-death, cascade, two-state and autoregulatory models
// of Secs. 3.1.1-3.1.3): the channels are the model's reactions in the order
// of its rates, and each
// entry of A(t)^T is formed from the state's coordinates inside the stage
// kernel, so a stage streams only the vectors.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace mjp {

constexpr int kRkB = 256;
constexpr int kRkMaxChannels = 8;
constexpr int kRkMaxBlocks = 2048;

struct RkOp {
    const int32_t* __restrict__ slice_off;
    const int32_t* __restrict__ col;
    const double* __restrict__ val;
    const uint8_t* __restrict__ ch;
};

struct RkG {
    double g[kRkMaxChannels];
};

// Block index for the grid-stride loops: workgroups are dispatched
// round-robin over the 8 XCDs, so renumber them (when the grid is a multiple
// of 8) to give each XCD one band of consecutive 256-row chunks per pass.  A
// row's neighbours (a grid line away, the rows its product gathers) then
// mostly lie in the same band and are served from that XCD's own L2 instead
// of being fetched again by the XCDs of the blocks next to it.
__device__ __forceinline__ int64_t rk_block() {
    const unsigned b = blockIdx.x, G = gridDim.x;
    return (G & 7u) ? (int64_t)b : (int64_t)((b & 7u) * (G >> 3) + (b >> 3));
}

// Row r of a stage once k = (xin A(t_s))_r is formed: FINAL: xout = x + h6
// (acc + k); otherwise xout = x + c_next k and acc = (first ? 0 : acc) + w k.
template <bool FINAL>
__device__ __forceinline__ void rk_stage_row(int64_t r, double k, const double* __restrict__ x,
                                             double* __restrict__ xout, double* __restrict__ acc, double c_next,
                                             double w, int first, double h6) {
    if constexpr (FINAL) {
        xout[r] = x[r] + h6 * (acc[r] + k);
    } else {
        xout[r] = x[r] + c_next * k;
        acc[r] = (first ? 0.0 : acc[r]) + w * k;
    }
}

// k = xin A(t_s) for each row, then rk_stage_row.
template <bool FINAL>
__global__ __launch_bounds__(kRkB) void k_rk_stage(RkOp op, RkG gv, const double* __restrict__ xin,
                                                   const double* __restrict__ x, double* __restrict__ xout,
                                                   double* __restrict__ acc, int64_t n, double c_next, double w,
                                                   int first, double h6) {
    __shared__ double gs[kRkMaxChannels];
    if (threadIdx.x < kRkMaxChannels) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < kRkMaxChannels; ++c)
            if (c == (int)threadIdx.x) v = gv.g[c];
        gs[threadIdx.x] = v;
    }
    __syncthreads();
    for (int64_t r = rk_block() * kRkB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kRkB) {
        const int64_t s = r >> 6;
        const int lane = (int)(r & 63);
        const int32_t b = op.slice_off[s] + lane;
        const int wdt = (op.slice_off[s + 1] - op.slice_off[s]) >> 6;
        double k = 0.0;
        int j = 0;
        for (; j + 4 <= wdt; j += 4) {  // four entries' indices, then their gathers
            int32_t c[4];
            double a[4], xv[4];
            int ch[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = op.col[b + (j + u) * 64];
                a[u] = op.val[b + (j + u) * 64];
                ch[u] = op.ch[b + (j + u) * 64];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = xin[c[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) k += gs[ch[u]] * a[u] * xv[u];
        }
        for (; j < wdt; ++j) {
            const int32_t e = b + j * 64;
            k += gs[op.ch[e]] * op.val[e] * xin[op.col[e]];
        }
        rk_stage_row<FINAL>(r, k, x, xout, acc, c_next, w, first, h6);
    }
}

// Stencil operator: the channels are the model's reactions in the order of
// its rates; births (and unbinding) that would leave the grid are dropped,
// as in the models' generators (conservative truncation).
//   birth-death / cascade, r = x1 + S1 x2 (birth-death: S2 = 1): 0 birth of
//     x1 (th0), 1 its death (th1 x1), 2 birth of x2 (th2 x1), 3 its death
//     (th3 x2);
//   two-state, r = n + S1 g (g = 0 active): 0 birth (th0, active), 1 death
//     (th1 n), 2 activation (th2, from inactive), 3 inactivation (th3);
//   autoregulatory, r = n_R + S1 n_P + S1 S2 g (S2 = N_P): 0 R birth (th0,
//     active), 1 P birth (th1 n_R), 2 R death (th2 n_R), 3 P death (th3 n_P),
//     4 unbinding inactive -> active + P (th4), 5 binding active + P ->
//     inactive (th5 n_P).
struct RkStencil {
    int32_t S1, S2;
    double th[6];  // 0 for channels the model lacks
};

// (xin A(t_s))_r for state r: the inflows from its neighbours, minus its
// exit rate; c[i] = g_i th_i, the stage's effective rates.
template <int MODEL>
__device__ __forceinline__ double rk_stencil_row(const RkStencil& m, const double* c, const double* __restrict__ xin,
                                                 int32_t r) {
    const uint32_t S1 = (uint32_t)m.S1;
    const uint32_t q = (uint32_t)r / S1, i1 = (uint32_t)r - q * S1;
    const double f1 = (double)i1;
    const bool up1 = i1 + 1 < S1;
    if constexpr (MODEL == MJP_MODEL_BD || MODEL == MJP_MODEL_CASCADE2) {
        const double f2 = (double)q;
        const bool up2 = (int32_t)q + 1 < m.S2;
        double k = -((up1 ? c[0] : 0.0) + c[1] * f1 + (up2 ? c[2] * f1 : 0.0) + c[3] * f2) * xin[r];
        if (i1 > 0) k += c[0] * xin[r - 1];
        if (up1) k += c[1] * (f1 + 1.0) * xin[r + 1];
        if (q > 0) k += c[2] * f1 * xin[r - (int32_t)S1];
        if (up2) k += c[3] * (f2 + 1.0) * xin[r + (int32_t)S1];
        return k;
    } else if constexpr (MODEL == MJP_MODEL_TWOSTATE) {
        const bool act = q == 0;
        double k = -((act && up1 ? c[0] : 0.0) + c[1] * f1 + (act ? c[3] : c[2])) * xin[r];
        if (act && i1 > 0) k += c[0] * xin[r - 1];
        if (up1) k += c[1] * (f1 + 1.0) * xin[r + 1];
        k += act ? c[2] * xin[r + (int32_t)S1] : c[3] * xin[r - (int32_t)S1];
        return k;
    } else {  // MJP_MODEL_AUTOREG
        const uint32_t NP = (uint32_t)m.S2, plane = S1 * NP;
        const uint32_t g = q / NP, p = q - g * NP;
        const bool act = g == 0, upp = p + 1 < NP;
        const double fp = (double)p;
        double k = -((act && up1 ? c[0] : 0.0) + (upp ? c[1] * f1 : 0.0) + c[2] * f1 + c[3] * fp +
                     (act ? c[5] * fp : (upp ? c[4] : 0.0))) * xin[r];
        if (act && i1 > 0) k += c[0] * xin[r - 1];                               // R birth
        if (p > 0) k += c[1] * f1 * xin[r - (int32_t)S1];                         // P birth
        if (up1) k += c[2] * (f1 + 1.0) * xin[r + 1];                             // R death
        if (upp) k += c[3] * (fp + 1.0) * xin[r + (int32_t)S1];                   // P death
        if (!act && upp) k += c[5] * (fp + 1.0) * xin[r - (int32_t)plane + (int32_t)S1];  // binding
        if (act && p > 0) k += c[4] * xin[r + (int32_t)plane - (int32_t)S1];     // unbinding
        return k;
    }
}

// k = xin A(t_s) from the stencil for each row, then rk_stage_row.
template <bool FINAL, int MODEL>
__global__ __launch_bounds__(kRkB) void k_rk_stage_stencil(RkStencil m, RkG gv, const double* __restrict__ xin,
                                                           const double* __restrict__ x, double* __restrict__ xout,
                                                           double* __restrict__ acc, int32_t n, double c_next,
                                                           double w, int first, double h6) {
    double c[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) c[i] = gv.g[i] * m.th[i];
    for (int32_t r = (int32_t)(rk_block() * kRkB + threadIdx.x); r < n; r += (int32_t)(gridDim.x * kRkB))
        rk_stage_row<FINAL>(r, rk_stencil_row<MODEL>(m, c, xin, r), x, xout, acc, c_next, w, first, h6);
}

__global__ void k_rk_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
    for (int64_t r = (int64_t)blockIdx.x * kRkB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kRkB) b[r] = a[r];
}

}  // namespace mjp

using namespace mjp;

struct mjp_rk4 {
    int device = 0;
    int64_t n = 0;
    int32_t C = 0;
    double dt_factor = 1.0;
    std::vector<std::vector<double>> knot_t, knot_g;  // per channel
    std::vector<std::vector<double>> absdiag;         // per channel |a^c_nn|
    bool stencil = false;                             // entries formed in the kernel (sten, model)
    int32_t model = 0;
    RkStencil sten{};
    DevBuf slice_off, col, val, ch;
    DevBuf x[2], s, t, acc;
};

namespace {

double sched(const std::vector<double>& kt, const std::vector<double>& kg, double t) {
    if (t <= kt.front()) return kg.front();
    if (t >= kt.back()) return kg.back();
    const size_t i = (size_t)(std::upper_bound(kt.begin(), kt.end(), t) - kt.begin());
    const double t0 = kt[i - 1], t1 = kt[i];
    return kg[i - 1] + (kg[i] - kg[i - 1]) * ((t - t0) / (t1 - t0));
}

// m = max over the knots of max_n sum_c g_c(t) |a^c_nn| (attained at a knot:
// max_n of functions linear in the g_c is convex in t between knots)
double rk_max_exit(const mjp_rk4* k) {
    std::vector<double> times;
    for (const auto& kt : k->knot_t) times.insert(times.end(), kt.begin(), kt.end());
    std::sort(times.begin(), times.end());
    times.erase(std::unique(times.begin(), times.end()), times.end());
    double best = 0.0;
    std::vector<double> g((size_t)k->C);
    for (double t : times) {
        for (int c = 0; c < k->C; ++c) g[(size_t)c] = sched(k->knot_t[(size_t)c], k->knot_g[(size_t)c], t);
        for (int64_t r = 0; r < k->n; ++r) {
            double e = 0.0;
            for (int c = 0; c < k->C; ++c) e += g[(size_t)c] * k->absdiag[(size_t)c][(size_t)r];
            best = std::max(best, e);
        }
    }
    return best;
}

}  // namespace

extern "C" {

void mjp_rk4_opts_default(mjp_rk4_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dt_factor = 1.0;
}

mjp_status mjp_rk4_create(int32_t n_channels, const mjp_csr* channels, const mjp_rk4_opts* opts, mjp_rk4** out) {
    clear_error();
    MJP_CHECK(out, MJP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    MJP_CHECK(opts, MJP_E_INVALID_ARG, "opts is NULL");
    MJP_CHECK(n_channels >= 1 && n_channels <= kRkMaxChannels, MJP_E_INVALID_ARG, "n_channels must be in [1, %d]",
              kRkMaxChannels);
    MJP_CHECK(channels, MJP_E_INVALID_ARG, "channels is NULL");
    MJP_CHECK(std::isfinite(opts->dt_factor) && opts->dt_factor > 0.0, MJP_E_INVALID_ARG,
              "dt_factor must be finite and > 0");
    const int32_t n = channels[0].n;
    std::vector<std::vector<double>> absdiag((size_t)n_channels);
    for (int c = 0; c < n_channels; ++c) {
        MJP_CHECK(channels[c].n == n, MJP_E_INVALID_ARG, "channel %d has %d states, channel 0 has %d", c,
                  channels[c].n, n);
        double m = 0.0;
        std::vector<double> diag;
        mjp_status st = check_generator_csr(&channels[c], 0, &m, &diag);
        if (st) return st;
        absdiag[(size_t)c].resize((size_t)n);
        for (int32_t r = 0; r < n; ++r) absdiag[(size_t)c][(size_t)r] = std::fabs(diag[(size_t)r]);
    }
    // merged A^T in pull form: output row m collects (source r, a^c_rm, c)
    std::vector<int32_t> cnt((size_t)n, 0);
    for (int c = 0; c < n_channels; ++c)
        for (int32_t r = 0; r < n; ++r)
            for (int32_t i = channels[c].row_ptr[r]; i < channels[c].row_ptr[r + 1]; ++i)
                cnt[(size_t)channels[c].col_idx[i]]++;
    const int32_t n_slices = (n + kSlice - 1) / kSlice;
    std::vector<int32_t> slice_off((size_t)n_slices + 1, 0);
    for (int32_t s = 0; s < n_slices; ++s) {
        int32_t w = 0;
        for (int32_t r = s * kSlice; r < std::min(n, (s + 1) * kSlice); ++r) w = std::max(w, cnt[(size_t)r]);
        const int64_t next = (int64_t)slice_off[(size_t)s] + (int64_t)w * kSlice;
        MJP_CHECK(next <= INT32_MAX, MJP_E_WORKSPACE, "operator too large");
        slice_off[(size_t)s + 1] = (int32_t)next;
    }
    const size_t total = (size_t)slice_off[(size_t)n_slices];
    std::vector<int32_t> hcol(total);
    std::vector<double> hval(total, 0.0);
    std::vector<uint8_t> hch(total, 0);
    for (int32_t s = 0; s < n_slices; ++s) {  // padding: own row, value 0
        const int32_t w = (slice_off[(size_t)s + 1] - slice_off[(size_t)s]) / kSlice;
        for (int32_t j = 0; j < w; ++j)
            for (int32_t l = 0; l < kSlice; ++l)
                hcol[(size_t)slice_off[(size_t)s] + (size_t)j * kSlice + l] = std::min(n - 1, s * kSlice + l);
    }
    std::vector<int32_t> fill((size_t)n, 0);
    for (int c = 0; c < n_channels; ++c)
        for (int32_t r = 0; r < n; ++r)
            for (int32_t i = channels[c].row_ptr[r]; i < channels[c].row_ptr[r + 1]; ++i) {
                const int32_t m = channels[c].col_idx[i];
                const int32_t s = m / kSlice, l = m % kSlice;
                const size_t at = (size_t)slice_off[(size_t)s] + (size_t)fill[(size_t)m] * kSlice + l;
                hcol[at] = r;
                hval[at] = channels[c].val[i];
                hch[at] = (uint8_t)c;
                fill[(size_t)m]++;
            }

    mjp_rk4* k = new (std::nothrow) mjp_rk4();
    MJP_CHECK(k, MJP_E_DEVICE, "out of host memory");
    auto bail = [&](mjp_status s) {
        mjp_rk4_destroy(k);
        return s;
    };
    if (hipGetDevice(&k->device) != hipSuccess) return bail(fail(MJP_E_DEVICE, "no HIP device available"));
    k->n = n;
    k->C = n_channels;
    k->dt_factor = opts->dt_factor;
    k->absdiag = std::move(absdiag);
    k->knot_t.assign((size_t)n_channels, std::vector<double>{0.0});
    k->knot_g.assign((size_t)n_channels, std::vector<double>{1.0});
    mjp_status st;
    const size_t vec = sizeof(double) * (size_t)n;
    if ((st = k->slice_off.reserve(sizeof(int32_t) * slice_off.size())) ||
        (st = k->col.reserve(sizeof(int32_t) * std::max<size_t>(total, 1))) ||
        (st = k->val.reserve(sizeof(double) * std::max<size_t>(total, 1))) ||
        (st = k->ch.reserve(std::max<size_t>(total, 1))) || (st = k->x[0].reserve(vec)) ||
        (st = k->x[1].reserve(vec)) || (st = k->s.reserve(vec)) || (st = k->t.reserve(vec)) ||
        (st = k->acc.reserve(vec)))
        return bail(st);
    auto up = [&](DevBuf& b, const void* h, size_t bytes) -> mjp_status {
        if (bytes) MJP_HIP(hipMemcpy(b.ptr, h, bytes, hipMemcpyHostToDevice));
        return MJP_OK;
    };
    if ((st = up(k->slice_off, slice_off.data(), sizeof(int32_t) * slice_off.size())) ||
        (st = up(k->col, hcol.data(), sizeof(int32_t) * total)) || (st = up(k->val, hval.data(), sizeof(double) * total)) ||
        (st = up(k->ch, hch.data(), total)))
        return bail(st);
    *out = k;
    return MJP_OK;
}

mjp_status mjp_rk4_create_stencil(const mjp_model* model, const mjp_rk4_opts* opts, mjp_rk4** out) {
    clear_error();
    MJP_CHECK(out, MJP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    MJP_CHECK(opts, MJP_E_INVALID_ARG, "opts is NULL");
    MJP_CHECK(std::isfinite(opts->dt_factor) && opts->dt_factor > 0.0, MJP_E_INVALID_ARG,
              "dt_factor must be finite and > 0");
    mjp_status st = check_model(model);
    if (st) return st;
    const int md = model->model;
    const int32_t S1 = model->dims[0], S2 = model->dims[1];  // birth-death and two-state: S2 = 1
    const int32_t n = md == MJP_MODEL_TWOSTATE ? 2 * S1 : md == MJP_MODEL_AUTOREG ? 2 * S1 * S2 : S1 * S2;
    const int C = md == MJP_MODEL_BD ? 2 : md == MJP_MODEL_AUTOREG ? 6 : 4;
    // |a^c_nn| per channel: the rate of reaction c out of state r, 0 where it would leave the grid
    std::vector<std::vector<double>> absdiag((size_t)C, std::vector<double>((size_t)n, 0.0));
    const double* th = model->theta;
    for (int32_t r = 0; r < n; ++r) {
        const int32_t i1 = r % S1, q = r / S1;
        const double f1 = (double)i1;
        if (md == MJP_MODEL_BD || md == MJP_MODEL_CASCADE2) {
            absdiag[0][(size_t)r] = i1 + 1 < S1 ? th[0] : 0.0;
            absdiag[1][(size_t)r] = th[1] * f1;
            if (C == 4) {
                absdiag[2][(size_t)r] = q + 1 < S2 ? th[2] * f1 : 0.0;
                absdiag[3][(size_t)r] = th[3] * (double)q;
            }
        } else if (md == MJP_MODEL_TWOSTATE) {
            const bool act = q == 0;
            absdiag[0][(size_t)r] = act && i1 + 1 < S1 ? th[0] : 0.0;
            absdiag[1][(size_t)r] = th[1] * f1;
            absdiag[2][(size_t)r] = act ? 0.0 : th[2];
            absdiag[3][(size_t)r] = act ? th[3] : 0.0;
        } else {
            const int32_t g = q / S2, p = q % S2;
            const bool act = g == 0, upp = p + 1 < S2;
            absdiag[0][(size_t)r] = act && i1 + 1 < S1 ? th[0] : 0.0;
            absdiag[1][(size_t)r] = upp ? th[1] * f1 : 0.0;
            absdiag[2][(size_t)r] = th[2] * f1;
            absdiag[3][(size_t)r] = th[3] * (double)p;
            absdiag[4][(size_t)r] = !act && upp ? th[4] : 0.0;
            absdiag[5][(size_t)r] = act ? th[5] * (double)p : 0.0;
        }
    }
    mjp_rk4* k = new (std::nothrow) mjp_rk4();
    MJP_CHECK(k, MJP_E_DEVICE, "out of host memory");
    auto bail = [&](mjp_status s) {
        mjp_rk4_destroy(k);
        return s;
    };
    if (hipGetDevice(&k->device) != hipSuccess) return bail(fail(MJP_E_DEVICE, "no HIP device available"));
    k->n = n;
    k->C = C;
    k->dt_factor = opts->dt_factor;
    k->absdiag = std::move(absdiag);
    k->knot_t.assign((size_t)C, std::vector<double>{0.0});
    k->knot_g.assign((size_t)C, std::vector<double>{1.0});
    k->stencil = true;
    k->model = md;
    k->sten.S1 = S1;
    k->sten.S2 = S2;
    for (int c = 0; c < 6; ++c) k->sten.th[c] = c < C ? th[c] : 0.0;
    const size_t vec = sizeof(double) * (size_t)n;
    if ((st = k->x[0].reserve(vec)) || (st = k->x[1].reserve(vec)) || (st = k->s.reserve(vec)) ||
        (st = k->t.reserve(vec)) || (st = k->acc.reserve(vec)))
        return bail(st);
    *out = k;
    return MJP_OK;
}

mjp_status mjp_rk4_set_schedule(mjp_rk4* k, int32_t channel, int32_t n_knots, const double* t_knots,
                                const double* g_knots) {
    clear_error();
    MJP_CHECK(k, MJP_E_INVALID_ARG, "handle is NULL");
    MJP_CHECK(channel >= 0 && channel < k->C, MJP_E_INVALID_ARG, "channel %d out of range", channel);
    MJP_CHECK(n_knots >= 1 && t_knots && g_knots, MJP_E_INVALID_ARG, "need >= 1 knot");
    for (int i = 0; i < n_knots; ++i) {
        MJP_CHECK(std::isfinite(t_knots[i]) && std::isfinite(g_knots[i]) && g_knots[i] >= 0.0, MJP_E_INVALID_ARG,
                  "knot %d: times and values must be finite, values >= 0", i);
        MJP_CHECK(i == 0 || t_knots[i] > t_knots[i - 1], MJP_E_INVALID_ARG, "knot times must increase");
    }
    k->knot_t[(size_t)channel].assign(t_knots, t_knots + n_knots);
    k->knot_g[(size_t)channel].assign(g_knots, g_knots + n_knots);
    return MJP_OK;
}

void mjp_rk4_destroy(mjp_rk4* k) {
    if (!k) return;
    int prev = 0;
    const bool restore = hipGetDevice(&prev) == hipSuccess;
    if (restore) (void)hipSetDevice(k->device);
    k->slice_off.release();
    k->col.release();
    k->val.release();
    k->ch.release();
    for (auto& b : k->x) b.release();
    k->s.release();
    k->t.release();
    k->acc.release();
    if (restore) (void)hipSetDevice(prev);
    delete k;
}

int32_t mjp_rk4_n(const mjp_rk4* k) { return k ? (int32_t)k->n : 0; }

mjp_status mjp_rk4_expv(mjp_rk4* k, const double* rho0_d, int32_t n_t, const double* t_h, double* out_d,
                        mjp_rk4_info* info_h, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(k, MJP_E_INVALID_ARG, "handle is NULL");
    MJP_CHECK(n_t >= 1, MJP_E_INVALID_ARG, "n_t must be >= 1");
    MJP_CHECK(t_h && rho0_d && out_d, MJP_E_INVALID_ARG, "null argument");
    for (int j = 0; j < n_t; ++j)
        MJP_CHECK(std::isfinite(t_h[j]) && t_h[j] >= 0.0, MJP_E_INVALID_ARG, "t[%d] must be finite and >= 0", j);
    int dev = 0;
    MJP_HIP(hipGetDevice(&dev));
    MJP_CHECK(dev == k->device, MJP_E_INVALID_ARG, "handle belongs to device %d, current device is %d", k->device, dev);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = k->n;
    const unsigned grid = (unsigned)std::min<int64_t>((n + kRkB - 1) / kRkB, kRkMaxBlocks);
    RkOp op{k->slice_off.as<int32_t>(), k->col.as<int32_t>(), k->val.as<double>(), k->ch.as<uint8_t>()};
    const double m = rk_max_exit(k);
    const double dt = m > 0.0 ? k->dt_factor / m : INFINITY;
    auto gset = [&](double t) {
        RkG g{};
        for (int c = 0; c < k->C; ++c) g.g[c] = sched(k->knot_t[(size_t)c], k->knot_g[(size_t)c], t);
        return g;
    };
    // one stage: k from xin with the stage's g, then the row update
    auto stage = [&](bool fin, const RkG& g, const double* xin, const double* x, double* xout, double c_next,
                     double w, int first, double h6) {
        double* ACCp = k->acc.as<double>();
        if (k->stencil) {
            const int32_t n32 = (int32_t)n;
#define MJP_RK_STENCIL(F, M)                                                                                    \
    hipLaunchKernelGGL((k_rk_stage_stencil<F, M>), dim3(grid), dim3(kRkB), 0, st, k->sten, g, xin, x, xout, ACCp, n32, \
                       c_next, w, first, h6)
            switch (k->model) {
                case MJP_MODEL_BD:
                case MJP_MODEL_CASCADE2:
                    if (fin) MJP_RK_STENCIL(true, MJP_MODEL_CASCADE2);
                    else MJP_RK_STENCIL(false, MJP_MODEL_CASCADE2);
                    break;
                case MJP_MODEL_TWOSTATE:
                    if (fin) MJP_RK_STENCIL(true, MJP_MODEL_TWOSTATE);
                    else MJP_RK_STENCIL(false, MJP_MODEL_TWOSTATE);
                    break;
                default:
                    if (fin) MJP_RK_STENCIL(true, MJP_MODEL_AUTOREG);
                    else MJP_RK_STENCIL(false, MJP_MODEL_AUTOREG);
                    break;
            }
#undef MJP_RK_STENCIL
        } else if (fin) {
            hipLaunchKernelGGL(k_rk_stage<true>, dim3(grid), dim3(kRkB), 0, st, op, g, xin, x, xout, ACCp, n, c_next, w,
                               first, h6);
        } else {
            hipLaunchKernelGGL(k_rk_stage<false>, dim3(grid), dim3(kRkB), 0, st, op, g, xin, x, xout, ACCp, n, c_next,
                               w, first, h6);
        }
    };

    std::vector<int> order((size_t)n_t);
    for (int j = 0; j < n_t; ++j) order[(size_t)j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return t_h[a] < t_h[b]; });
    int cur = 0;
    double* X[2] = {k->x[0].as<double>(), k->x[1].as<double>()};
    double* S = k->s.as<double>();
    double* T = k->t.as<double>();
    hipLaunchKernelGGL(k_rk_copy, dim3(grid), dim3(kRkB), 0, st, rho0_d, X[0], n);
    double tau = 0.0;
    int64_t steps = 0;
    for (int idx : order) {
        const double te = t_h[idx];
        while (te - tau > 0.0 && m > 0.0) {
            const double h = std::min(dt, te - tau);
            const bool lands = h == te - tau;
            const double* x = X[cur];
            double* xn = X[cur ^ 1];
            const RkG g0 = gset(tau), gh = gset(tau + 0.5 * h), g1 = gset(tau + h);
            stage(false, g0, x, x, S, 0.5 * h, 1.0, 1, 0.0);
            stage(false, gh, S, x, T, 0.5 * h, 2.0, 0, 0.0);
            stage(false, gh, T, x, S, h, 2.0, 0, 0.0);
            stage(true, g1, S, x, xn, 0.0, 0.0, 0, h / 6.0);
            cur ^= 1;
            tau = lands ? te : tau + h;
            ++steps;
        }
        hipLaunchKernelGGL(k_rk_copy, dim3(grid), dim3(kRkB), 0, st, (const double*)X[cur], out_d + (size_t)idx * n, n);
    }
    MJP_HIP(hipGetLastError());
    if (info_h) {
        std::memset(info_h, 0, sizeof(*info_h));
        info_h->m = m;
        info_h->dt = dt;
        info_h->steps = steps;
    }
    return MJP_OK;
}

}  // extern "C"
