// Batched snapshot log-likelihoods (Sec. 2.1.2):
//   loglik[b] = sum_i count_i log rho_b(T_{j_i})_{s_i}
// for B parameter draws of a built-in model, each on its own grid, in one
// persistent launch.
//
//   k_ll_prep   one thread per (item, time): Omega from theta and the grid,
//               then the jump window [L, K] of W = Omega T by walking out from
//               the Poisson mode with the ratio recurrence (FP64); K is the
//               first jump whose geometric bound on the right tail is below
//               tol/4, L the last whose bound on the left tail is; the window
//               weight sum gives the residual lumped at K (Algorithm 2).
//   k_ll_order  one block: items grouped by size class (states <= 5120,
//               10240, 20480, 40000), longest first (cost K_max * N) inside
//               a class; writes the class offsets.
//   k_ll_main   one launch per size class, each instance a (model, shape):
//               shape = T threads x C cells per thread, with exactly the LDS
//               of T*C states, so small shapes let several workgroups share a
//               CU.  Workgroups pull the class's items from an atomic queue.
//               The whole state vector of an item sits in LDS; each thread
//               owns cells m = tid + i*T; a jump is "compute the new values of
//               my cells into registers, barrier, write back, barrier".  The
//               shape per class is a default or the one mjp_loglik_tune
//               measured fastest on the caller's batch.  Only observed states are
//               accumulated (Kahan, FP32), one observation record per thread;
//               the per-time weights are formed in FP64 log space by one
//               thread per time.  The final sum of count * log p is FP64.
#include <algorithm>
#include <cfloat>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "gridsync.h"
#include "internal.h"

namespace mjp {

mjp_status check_opts(const mjp_opts* o);

constexpr int kLLMaxStates = 40000;            // 160,000 B of LDS
constexpr int kLLMaxTimes = 64;
constexpr int kLLRecPerThread = 4;
constexpr int kLLMaxRecords = 1024 * kLLRecPerThread;
constexpr int kLLMaxSort = 16384;
constexpr int kLLExtraLds = 3584;             // weights, window table, reduction scratch

// size classes of items (states S1*S2) and the launch shapes
constexpr int kLLClasses = MJP_LL_CLASSES;
constexpr int kLLClassCap[kLLClasses] = {5120, 10240, 20480, kLLMaxStates};
__host__ __device__ inline int ll_class(int64_t n) { return n <= 5120 ? 0 : (n <= 10240 ? 1 : (n <= 20480 ? 2 : 3)); }

struct LLShape {
    int T, C;  // threads per workgroup, cells per thread
};
constexpr LLShape kLLShapes[] = {{1024, 40}, {512, 80}, {1024, 20}, {512, 40}, {256, 80}, {1024, 10}, {512, 20},
                                 {256, 40},  {1024, 5}, {512, 10},  {256, 20}, {768, 53}, {768, 27}};
constexpr int kLLNumShapes = (int)(sizeof(kLLShapes) / sizeof(kLLShapes[0]));
static_assert(kLLNumShapes <= MJP_LL_MAX_SHAPES, "shape table larger than the report");
constexpr int kLLDefaultShape[kLLClasses] = {8, 5, 2, 0};  // T = 1024, tightest C
constexpr int ll_cap(int T, int C) { return T * C < kLLMaxStates ? T * C : kLLMaxStates; }

// Column kernel (cascade items; k_ll_col below).  Its item loop once
// popped the queue under "if (tid == 0)", which the compiler folded into
// the loop's back edge so that the workgroup repeated an item for ever (see
// queue_pop); kColEnabled switches it off again if needed.  1024
// threads, 62 real lanes per wave (lanes 0 and 63 are ghost lanes), so 992
// column segments per workgroup; an item's class is the register template C
// that holds its segment length.  Queue and class-offset entries: the
// column classes first, then the four size classes of the cell kernel.
constexpr int kColT = 1024;
constexpr int kColReal = 62;
constexpr int kColLanes = kColReal * (kColT / 64);
constexpr int kColClasses = 9;
// (50: a 200-row column in four segments fits the mirror at stride 201,
// where 56-row segments would pad it to 225)
constexpr int kColCs[kColClasses] = {8, 16, 24, 32, 40, 48, 50, 56, 64};
constexpr bool kColEnabled = true;

// Items above one workgroup's LDS (cascade and birth-death, S1*S2 >
// kLLMaxStates) run in clusters of kClG workgroups (k_ll_cluster below):
// each owns a contiguous range of at most kClOwn states and exchanges its
// boundary rows with its neighbours every kClJumps jumps (every jump where
// the item does not allow that).  Their queue class follows the cell
// kernel's.
constexpr int kClT = 1024;
constexpr int kClC = 32;
constexpr int kClOwn = kClT * kClC;        // states one workgroup owns at most
constexpr int kClG = 4;                    // workgroups per item
constexpr int kClReachMax = 1024;          // S1 of a cascade item at most
constexpr int kClJumps = 4;                // jumps per exchange where an item allows (else 1)
constexpr int kClSlot = 2048;              // states per exchange slot: reach, or kClJumps x reach
constexpr int kClMaxStates = kClG * kClOwn;
constexpr int kClClass = kColClasses + kLLClasses;
constexpr int kAllClasses = kClClass + 1;

// Segments of an item (S1 columns, S2 rows) for the column kernel: nseg
// segments of len = kColCs[class] consecutive rows (the register template,
// the smallest that needs at most 992 lanes, nseg * S1 <= 992).  The LDS
// mirror is column-major with column stride S2p = (nseg * len) | 1 >= S2
// (rows S2 and beyond hold zeros; an odd stride puts consecutive columns in
// different banks).  False if it does not fit (S1 > 992, more than 64 rows
// per segment, or a mirror larger than kColMirror).
constexpr int kColMirror = 40256;  // floats of the mirror (the rest of 160 KB holds weights and tables)
__host__ __device__ inline bool col_geom(int S1, int S2, int& cls, int& nseg, int& len, int& S2p) {
    if (S1 < 1 || S2 < 1 || S1 > kColLanes || (int64_t)S1 * S2 > kLLMaxStates) return false;
    const int ns = kColLanes / S1 < S2 ? kColLanes / S1 : S2;
    const int need = (S2 + ns - 1) / ns;  // fewest rows per segment
    cls = 0;
    while (cls < kColClasses && kColCs[cls] < need) ++cls;
    if (cls == kColClasses) return false;
    len = kColCs[cls];
    nseg = (S2 + len - 1) / len;
    S2p = (nseg * len) | 1;
    return (int64_t)S1 * S2p <= kColMirror;
}
// mirror entries the column kernel of class cc holds in LDS (every lane's
// segment plus one padding row per column)
constexpr int col_cap(int cc) {
    return kColLanes * (kColCs[cc] + 1) < kColMirror ? kColLanes * (kColCs[cc] + 1) : kColMirror;
}

struct LLWin {     // per (item, time)
    double W;
    double lastw;  // w_K + residual (lumping) or w_K
    double aw;     // w_L: the anchor of the sweep's weight recurrence
    int32_t L, K;
};
// Weights in the sweeps: w_L = aw from the window (formed by k_ll_prep's
// walk from the mode), then w_k = w_{k-1} W / k in FP64 -- one division per
// jump instead of a log and an exp.  The recurrence's relative rounding grows
// by about 2.2e-16 per jump, below 1e-11 over any window here.  Under the
// paper's K rule (L = 0) at W > 667 the weights of the first jumps are below
// FP64's range; the window then starts at the first k whose weight is at
// least kWeightFloor (every weight skipped is below 1e-290).
constexpr double kWeightFloor = 1e-290;
// the part of a window every thread of a sweep reads, kept in LDS (the
// anchor stays in the register of the thread that forms the time's weights)
struct LLWinL {
    double W, lastw;
    int32_t L, K;
};
__device__ __forceinline__ LLWinL ll_win_lds(const LLWin& w) { return LLWinL{w.W, w.lastw, w.L, w.K}; }
// a time's weight at jump k, from the previous jump's (cur)
__device__ __forceinline__ double ll_weight_step(int k, double W, int L, double aw, double cur) {
    if (k == L) return aw;
    return k > L ? cur * (W / (double)k) : 0.0;
}

struct LLRecord {  // per observation record
    int32_t t, x1, x2, count;
};

struct LLArgs {
    const double* __restrict__ theta;   // [B][4]
    const int32_t* __restrict__ dims;   // [B][2]
    const double* __restrict__ T;       // [n_t]
    const LLRecord* __restrict__ rec;   // [n_rec]
    LLWin* __restrict__ win;            // [B][n_t]
    float* __restrict__ cost;           // [B]
    int32_t* __restrict__ order;        // [B]
    unsigned* __restrict__ queue;       // [kLLClasses]
    int32_t* __restrict__ cls_off;      // [kLLClasses + 1] class ranges of order[]
    double* __restrict__ loglik;        // [B]
    mjp_info* __restrict__ info;        // [B] or null
    const int32_t* __restrict__ kobs;   // jump mode: [B][n_rec] jump count of each observation
    double* __restrict__ phi;           // jump mode: [B][n_rec] log p(s_i | k_i, theta)
    double* __restrict__ omega_out;     // jump mode: [B] Omega_theta, or null
    const uint8_t* __restrict__ active; // [B] or null: items with 0 are skipped (outputs untouched)
    int32_t B, n_t, n_rec, model, x0_1, x0_2;
    int32_t use_col;                    // cascade items that fit go to the column kernel
    int32_t use_cluster;                // cascade/birth-death items above kLLMaxStates go to clusters
    double omega_factor, tol;
    int32_t k_rule, lump, renorm_every;
    int32_t one_jump;                   // clusters exchange every jump (opts->variant MJP_VARIANT_PERSISTENT_ONEJUMP)
    int64_t k_cap;
};

// theta stride and parameter count of a model's draws
__host__ __device__ inline int ll_stride(int model) { return model == MJP_MODEL_AUTOREG ? 6 : 4; }
__host__ __device__ inline int ll_params(int model) {
    return model == MJP_MODEL_BD ? 2 : (model == MJP_MODEL_AUTOREG ? 6 : 4);
}
// grid of an item as (S1, S2): BD {N, 1}; cascade {S1, S2}; two-state
// {N_R, 2} (second coordinate = gene state); autoregulatory {N_R, 2 N_P}
// (second coordinate = n_P + N_P g)
__device__ inline void ll_grid(int model, const int32_t* d, int& S1, int& S2) {
    S1 = d[0];
    S2 = model == MJP_MODEL_BD ? 1 : (model == MJP_MODEL_TWOSTATE ? 2 : (model == MJP_MODEL_AUTOREG ? 2 * d[1] : d[1]));
}

// max_n |a_nn| under conservative truncation; exits grow with every count
// except for births blocked at a cap, so the last two values of each count
// hold the maximum
__device__ double ll_max_exit(int model, const double* th, const int32_t* d) {
    double best = 0.0;
    if (model == MJP_MODEL_BD) {
        const int S1 = d[0];
        for (int n = max(0, S1 - 2); n < S1; ++n)
            best = fmax(best, ((n + 1 < S1) ? th[0] : 0.0) + th[1] * n);
    } else if (model == MJP_MODEL_CASCADE2) {
        const int S1 = d[0], S2 = d[1];
        for (int n2 = max(0, S2 - 2); n2 < S2; ++n2)
            for (int n1 = max(0, S1 - 2); n1 < S1; ++n1)
                best = fmax(best, ((n1 + 1 < S1) ? th[0] : 0.0) + th[1] * n1 + ((n2 + 1 < S2) ? th[2] * n1 : 0.0) +
                                      th[3] * n2);
    } else if (model == MJP_MODEL_TWOSTATE) {
        const int NR = d[0];
        for (int r = max(0, NR - 2); r < NR; ++r) {
            best = fmax(best, ((r + 1 < NR) ? th[0] : 0.0) + th[1] * r + th[3]);  // active
            best = fmax(best, th[1] * r + th[2]);                                 // inactive
        }
    } else {
        const int NR = d[0], NP = d[1];
        for (int p = max(0, NP - 2); p < NP; ++p)
            for (int r = max(0, NR - 2); r < NR; ++r) {
                const double common = ((p + 1 < NP) ? th[1] * r : 0.0) + th[2] * r + th[3] * p;
                best = fmax(best, common + ((r + 1 < NR) ? th[0] : 0.0) + th[5] * p);  // active
                best = fmax(best, common + ((p + 1 < NP) ? th[4] : 0.0));              // inactive
            }
    }
    return best;
}

__global__ void k_ll_prep(LLArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < kAllClasses) a.queue[idx] = 0u;
    if (idx >= a.B * a.n_t) return;
    const int b = idx / a.n_t, j = idx - b * a.n_t;
    if (a.active && !a.active[b]) return;
    const double* th = a.theta + ll_stride(a.model) * (int64_t)b;
    bool bad_theta = false;
    for (int i = 0; i < ll_params(a.model); ++i) bad_theta |= !(th[i] >= 0.0) || isinf(th[i]);
    const double omega = bad_theta ? 0.0 : a.omega_factor * ll_max_exit(a.model, th, a.dims + 2 * b);
    const double W = bad_theta ? NAN : omega * a.T[j];
    LLWin w;
    w.W = W;
    w.aw = 0.0;
    if (W == 0.0) {
        w.L = w.K = 0;
        w.lastw = 1.0;
        w.aw = 1.0;  // w_0 = 1, later weights W^k / k! = 0
    } else if (!(W > 0.0) || !(W < 1e9) || W > (double)a.k_cap) {
        // non-finite or enormous rates: K >= floor(W) already exceeds the cap
        w.L = 0;
        w.K = -1;
        w.lastw = 0.0;
        w.W = isfinite(W) ? W : 0.0;
    } else {
        const double eps = a.tol / 4.0;
        const double mode = floor(W);
        const double wm = exp(-W + mode * log(W) - lgamma(mode + 1.0));
        // right end
        double k = mode, wk = wm, sum = wm;
        int64_t K;
        if (a.k_rule == MJP_K_PAPER) {
            K = (int64_t)floor(W + 6.0 * sqrt(W)) + 1;
            while (k < (double)K) { wk = wk * W / (k + 1.0); k += 1.0; sum += wk; }
        } else {
            const double kstop = (double)a.k_cap + 1.0;  // bounded walk: past the cap the item is rejected
            while (k < kstop) {
                const double wn = wk * W / (k + 1.0);
                const double q = W / (k + 2.0);
                if (wn / (1.0 - q) <= eps) break;
                wk = wn;
                k += 1.0;
                sum += wk;
            }
            K = (int64_t)k;
        }
        const double wK = wk;
        // left end; the window starts at the smallest k walked whose weight
        // is at least kWeightFloor (the tolerance rule's L always qualifies)
        int64_t L;
        k = mode;
        wk = wm;
        double ka = mode, wa = wm;
        if (a.k_rule == MJP_K_PAPER) {
            while (k > 0.0) {
                wk = wk * k / W;
                k -= 1.0;
                sum += wk;
                if (wk >= kWeightFloor) { ka = k; wa = wk; }
            }
        } else {
            while (k > 0.0) {
                const double wp = wk * k / W;
                const double q = (k - 1.0) / W;
                if (wp / (1.0 - q) <= eps) break;
                wk = wp;
                k -= 1.0;
                sum += wk;
                if (wk >= kWeightFloor) { ka = k; wa = wk; }
            }
        }
        L = (int64_t)ka;
        w.aw = wa;
        const double resid = 1.0 - sum;
        w.K = (int32_t)min<int64_t>(K, (int64_t)INT32_MAX / 2);
        w.L = (int32_t)L;
        w.lastw = wK + (a.lump ? resid : 0.0);
        if (K > a.k_cap) w.K = -1;  // marks the item as over the cap
    }
    a.win[(int64_t)b * a.n_t + j] = w;
}

// Jump mode (J-MJP state probabilities): one window per item whose K is
// the largest jump count of its observations; an item with a count below 0
// or above k_cap gets K = -1 (rejected like an item over the cap).
__global__ void k_jp_prep(LLArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < kAllClasses) a.queue[b] = 0u;
    if (b >= a.B) return;
    int64_t kmax = 0;
    bool bad = false;
    for (int r = 0; r < a.n_rec; ++r) {
        const int32_t k = a.kobs[(int64_t)b * a.n_rec + r];
        bad |= k < 0 || (int64_t)k > a.k_cap;
        kmax = max(kmax, (int64_t)k);
    }
    LLWin w;
    w.W = 0.0;
    w.lastw = 0.0;
    w.aw = 0.0;
    w.L = 0;
    w.K = bad ? -1 : (int32_t)kmax;
    a.win[b] = w;
}

// queue class of an item: a column class when the column kernel takes it,
// else kColClasses + its size class
__device__ inline int ll_item_class(const LLArgs& a, int S1, int S2) {
    // (a.use_col is set only for cascade items with at most kColT records)
    const int64_t n = (int64_t)S1 * S2;
    if (a.use_cluster && n > kLLMaxStates && n <= kClMaxStates &&
        (a.model == MJP_MODEL_BD || (a.model == MJP_MODEL_CASCADE2 && S1 <= kClReachMax)))
        return kClClass;
    int cc, ns, len, S2p;
    if (a.use_col && col_geom(S1, S2, cc, ns, len, S2p) && (int64_t)S1 * S2p <= col_cap(cc)) return cc;
    return kColClasses + ll_class((int64_t)S1 * S2);
}

// cost of each item (max K over its times times its states), its queue
// class, then the items grouped by class (ascending) and longest-first inside
// a class; cls_off[c] .. cls_off[c+1] is class c's range of order[]
__global__ void k_ll_order(LLArgs a) {
    extern __shared__ unsigned long long keys[];
    __shared__ int cnt[kAllClasses], cur[kAllClasses];
    const int B = a.B;
    int P = 1;
    while (P < B) P <<= 1;
    const bool sort = P <= kLLMaxSort;
    if (threadIdx.x < kAllClasses) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < (sort ? P : B); b += blockDim.x) {
        unsigned long long key = ~0ull;  // padding and skipped items sort last, outside every class
        if (b < B && (!a.active || a.active[b])) {
            int32_t kmax = 0;
            for (int j = 0; j < a.n_t; ++j) kmax = max(kmax, a.win[(int64_t)b * a.n_t + j].K);
            int S1, S2;
            ll_grid(a.model, a.dims + 2 * b, S1, S2);
            const int cls = ll_item_class(a, S1, S2);
            if (cls == kClClass && a.loglik) a.loglik[b] = NAN;  // until its cluster finishes it
            atomicAdd(&cnt[cls], 1);
            const float c = fmaxf((float)(kmax + 1) * (float)S1 * (float)S2, 0.f);
            a.cost[b] = c;
            // class (4 bits), then descending cost (the inverted top 29 of
            // the 31 bits of a non-negative float), then the item (31 bits)
            key = ((unsigned long long)cls << 60) |
                  ((unsigned long long)((~__float_as_uint(c) & 0x7fffffffu) >> 2) << 31) | (unsigned)b;
        }
        if (sort) keys[b] = key;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int at = 0;
        for (int c = 0; c < kAllClasses; ++c) {
            a.cls_off[c] = at;
            cur[c] = at;
            at += cnt[c];
        }
        a.cls_off[kAllClasses] = at;
    }
    __syncthreads();
    if (!sort) {  // too many items to sort in LDS: grouped by class only
        for (int b = threadIdx.x; b < B; b += blockDim.x) {
            if (a.active && !a.active[b]) continue;
            int S1, S2;
            ll_grid(a.model, a.dims + 2 * b, S1, S2);
            a.order[atomicAdd(&cur[ll_item_class(a, S1, S2)], 1)] = b;
        }
        return;
    }
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int jx = i ^ stride;
                if (jx > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long u = keys[i], v = keys[jx];
                    if ((u > v) == up) { keys[i] = v; keys[jx] = u; }
                }
            }
            __syncthreads();
        }
    }
    for (int b = threadIdx.x; b < B; b += blockDim.x) a.order[b] = (int32_t)(keys[b] & 0x7fffffffu);
}

template <int T>
__device__ __forceinline__ double ll_block_sum(double v, double* scratch) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < T / 64; ++i) s += scratch[i];  // same order in every thread
    __syncthreads();
    return s;
}

// Rates of an item divided by Omega (FP32), and the number of P levels of
// the autoregulatory model.
struct LLCoef {
    float c[6];
    int NP;
};

// New value of cell m = i1 + S1 i2 after one jump (pull form y_m = sum_n
// rho_n b_nm).  The diagonal of B is 1 minus the FP64 sum of the state's
// FP32 exit coefficients, the same numbers its neighbours pull, held as an
// FP32 pair hi + lo so the row sums to 1 to ~1e-16.
template <int MODEL>
__device__ __forceinline__ float ll_cell(const float* rho, int m, int i1, int i2, int S1, int S2, const LLCoef& k) {
    const float f1 = (float)i1;
    if constexpr (MODEL == MJP_MODEL_BD || MODEL == MJP_MODEL_CASCADE2) {
        const float b1 = k.c[0], d1 = k.c[1], b2 = k.c[2], d2 = k.c[3];
        const float f2 = (float)i2;
        const float o_b1 = (i1 + 1 < S1) ? b1 : 0.f;
        const float o_b2 = (i2 + 1 < S2) ? b2 * f1 : 0.f;
        float dh, dl;
        diag_pair(1.0 - (((double)o_b1 + (double)(d1 * f1)) + ((double)o_b2 + (double)(d2 * f2))), dh, dl);
        float y = fmaf(dh, rho[m], dl * rho[m]);
        if (i1 > 0) y = fmaf(b1, rho[m - 1], y);
        if (i1 + 1 < S1) y = fmaf(d1 * (f1 + 1.f), rho[m + 1], y);
        if (i2 > 0) y = fmaf(b2 * f1, rho[m - S1], y);
        if (i2 + 1 < S2) y = fmaf(d2 * (f2 + 1.f), rho[m + S1], y);
        return y;
    } else if constexpr (MODEL == MJP_MODEL_TWOSTATE) {
        // i1 = n_R, i2 = gene state (0 active); c = beta, gamma, l_act, l_ina
        const float be = k.c[0], ga = k.c[1], la = k.c[2], li = k.c[3];
        const bool act = i2 == 0;
        const float o_b = (act && i1 + 1 < S1) ? be : 0.f;
        const float o_s = act ? li : la;
        float dh, dl;
        diag_pair(1.0 - (((double)o_b + (double)(ga * f1)) + (double)o_s), dh, dl);
        float y = fmaf(dh, rho[m], dl * rho[m]);
        if (act && i1 > 0) y = fmaf(be, rho[m - 1], y);
        if (i1 + 1 < S1) y = fmaf(ga * (f1 + 1.f), rho[m + 1], y);
        y = act ? fmaf(la, rho[m + S1], y) : fmaf(li, rho[m - S1], y);
        return y;
    } else {
        // i1 = n_R, i2 = n_P + NP g; c = beta_R, beta_P, gamma_R, gamma_P, l_act, l_ina
        const int NP = k.NP;
        const bool act = i2 < NP;
        const int p = act ? i2 : i2 - NP;
        const int plane = S1 * NP;
        const float fp = (float)p;
        const float o_bR = (act && i1 + 1 < S1) ? k.c[0] : 0.f;
        const float o_bP = (p + 1 < NP) ? k.c[1] * f1 : 0.f;
        const float o_sw = act ? k.c[5] * fp : ((p + 1 < NP) ? k.c[4] : 0.f);
        float dh, dl;
        diag_pair(1.0 - ((((double)o_bR + (double)o_bP) + ((double)(k.c[2] * f1) + (double)(k.c[3] * fp))) +
                         (double)o_sw),
                  dh, dl);
        float y = fmaf(dh, rho[m], dl * rho[m]);
        if (act && i1 > 0) y = fmaf(k.c[0], rho[m - 1], y);               // R birth from n_R - 1
        if (p > 0) y = fmaf(k.c[1] * f1, rho[m - S1], y);                 // P birth from n_P - 1
        if (i1 + 1 < S1) y = fmaf(k.c[2] * (f1 + 1.f), rho[m + 1], y);    // R death from n_R + 1
        if (p + 1 < NP) y = fmaf(k.c[3] * (fp + 1.f), rho[m + S1], y);    // P death from n_P + 1
        if (!act && p + 1 < NP) y = fmaf(k.c[5] * (fp + 1.f), rho[m - plane + S1], y);  // binding
        if (act && p > 0) y = fmaf(k.c[4], rho[m + plane - S1], y);       // unbinding
        return y;
    }
}

// JUMP: the J-MJP state probabilities (Method #2's algorithm): no weights;
// observation i records log rho_{k_i} at its state when the sweep reaches its
// own jump count k_i (one window per item, n_t = 1).
// Next slot of a work queue for the whole workgroup, with no branch: every
// thread adds (tid == 0) to the counter and each wave stores its first
// lane's old value in its own LDS word; wave 0's word is thread 0's slot.
// A pop written as "if (tid == 0) slot = atomicAdd(...)" at the top of an
// item loop lets the compiler fold that loop-invariant branch into the
// loop's back edge: the loop becomes a nest in which thread 0 alone goes
// round the pop while the other lanes of wave 0 go straight back to the
// barrier, so the workgroup passes the barrier without the pop and repeats
// its last item for ever.
__device__ __forceinline__ int queue_pop(unsigned* q, int* wslot) {
    const unsigned v = atomicAdd(q, threadIdx.x == 0 ? 1u : 0u);
    wslot[threadIdx.x >> 6] = (int)__builtin_amdgcn_readfirstlane(v);
    __syncthreads();
    const int r = __builtin_amdgcn_readfirstlane(wslot[0]);
    __syncthreads();
    return r;
}

template <int MODEL, int T, int C, bool JUMP = false>
__global__ __launch_bounds__(T) void k_ll_main(LLArgs a, int cls) {
    constexpr int CAP = ll_cap(T, C);  // states this shape holds (a multiple of 2)
    extern __shared__ char lds[];
    float* rho = reinterpret_cast<float*>(lds);                          // [CAP]
    double* wbuf = reinterpret_cast<double*>(lds + sizeof(float) * CAP);  // [2][kLLMaxTimes]
    double* scratch = wbuf + 2 * kLLMaxTimes;                                      // [16]
    LLWinL* win = reinterpret_cast<LLWinL*>(scratch + 16);                         // [kLLMaxTimes]
    __shared__ int pop_sh[T / 64];
    __shared__ unsigned flag_sh;
    const int tid = threadIdx.x;

    const int first = a.cls_off[cls], last = a.cls_off[cls + 1];
    while (true) {
        const int slot = first + queue_pop(a.queue + cls, pop_sh);
        if (slot >= last) break;
        const int b = a.order[slot];
        const double* th = a.theta + ll_stride(MODEL) * (int64_t)b;
        int S1, S2;
        ll_grid(MODEL, a.dims + 2 * b, S1, S2);
        double w_aw = 0.0;  // the anchor weight of this thread's time (threads tid < n_t)
        if (tid < a.n_t) {
            const LLWin wg = a.win[(int64_t)b * a.n_t + tid];
            win[tid] = ll_win_lds(wg);
            w_aw = wg.aw;
        }
        if (tid == 0) flag_sh = 0u;
        __syncthreads();
        unsigned flags = 0;
        int32_t Kmax = 0, Lmin = INT32_MAX;
        bool over = false;
        for (int j = 0; j < a.n_t; ++j) {
            const int Kj = win[j].K;
            if (Kj < 0) over = true;
            Kmax = max(Kmax, Kj);
            Lmin = min(Lmin, win[j].L);
        }
        const int64_t N64 = (int64_t)S1 * S2;
        double omega = a.omega_factor * ll_max_exit(MODEL, th, a.dims + 2 * b);
        if (over || S1 < 1 || S2 < 1 || N64 > CAP) {
            if constexpr (JUMP) {
                for (int r = tid; r < a.n_rec; r += T) a.phi[(int64_t)b * a.n_rec + r] = -INFINITY;
                if (tid == 0 && a.omega_out) a.omega_out[b] = omega;
            }
            if (tid == 0) {
                if (!JUMP) a.loglik[b] = -INFINITY;
                if (a.info) {
                    mjp_info inf{};
                    inf.omega = omega;
                    inf.flags = over ? MJP_FLAG_K_LIMIT : MJP_FLAG_OUT_OF_GRID;
                    a.info[b] = inf;
                }
            }
            continue;
        }
        const int N = (int)N64;
        const double om = omega > 0.0 ? omega : 1.0;
        LLCoef kc;
#pragma unroll
        for (int i = 0; i < 6; ++i) kc.c[i] = i < ll_params(MODEL) ? (float)(th[i] / om) : 0.f;
        kc.NP = MODEL == MJP_MODEL_AUTOREG ? a.dims[2 * b + 1] : 1;

        // owned cells, their coordinates advance by T = q*S1 + r per step
        const int qT = T / S1, rT = T - qT * S1;
        // rho(0) = point mass at x0 (if on the grid); for the two-state model
        // x0 = (n_R, gene state), for the autoregulatory one (n_R, n_P), active
        const int x0lim2 = MODEL == MJP_MODEL_AUTOREG ? kc.NP : S2;
        const int x0 = (a.x0_1 < S1 && a.x0_2 < x0lim2) ? a.x0_1 + S1 * a.x0_2 : -1;
        for (int m = tid; m < N; m += T) rho[m] = (m == x0) ? 1.f : 0.f;

        // observation records of this thread
        // an observed state; for the two gene-state models it is observed
        // without the gene state, so the record sums cells rm and rm + hid
        constexpr bool kHidden = MODEL == MJP_MODEL_TWOSTATE || MODEL == MJP_MODEL_AUTOREG;
        const int hid = MODEL == MJP_MODEL_TWOSTATE ? S1 : S1 * kc.NP;
        const int lim2 = MODEL == MJP_MODEL_TWOSTATE ? 1 : (MODEL == MJP_MODEL_AUTOREG ? kc.NP : S2);
        int rm[kLLRecPerThread], rt[kLLRecPerThread];
        float rs[kLLRecPerThread], rc[kLLRecPerThread];
#pragma unroll
        for (int u = 0; u < kLLRecPerThread; ++u) {
            const int r = tid + u * T;
            rm[u] = -2;
            rt[u] = 0;
            rs[u] = 0.f;
            rc[u] = 0.f;
            if (r < a.n_rec) {
                const LLRecord R = a.rec[r];
                rt[u] = JUMP ? a.kobs[(int64_t)b * a.n_rec + r] : R.t;  // jump mode: the jump count
                rm[u] = (R.x1 < S1 && R.x2 < lim2) ? R.x1 + S1 * R.x2 : -1;
                if (rm[u] < 0) {
                    flags |= MJP_FLAG_OUT_OF_GRID;
                    if (JUMP) a.phi[(int64_t)b * a.n_rec + r] = -INFINITY;
                }
            }
        }
        if (tid < a.n_t) wbuf[tid] = 0.0;
        __syncthreads();
        if (x0 < 0) flags |= MJP_FLAG_OUT_OF_GRID;

        const int i1_0 = tid % S1, i2_0 = tid / S1;
        double scale = 1.0;
        const int m_renorm = a.renorm_every;
        double wcur = 0.0;  // this time's weight at the current jump (threads tid < n_t)
        for (int k = 0; k <= Kmax; ++k) {
            // weight of jump k for each time (FP64, the recurrence from w_L)
            if (!JUMP && tid < a.n_t) {
                wcur = ll_weight_step(k, win[tid].W, win[tid].L, w_aw, wcur);
                wbuf[(k & 1) * kLLMaxTimes + tid] = wcur;
            }
            if (k > 0) {
                float nv[C];
                int i1 = i1_0, i2 = i2_0, mb = tid;
                // opaque to the optimiser: stops it hoisting C cells' worth of
                // addresses and predicates out of the jump loop (which spills)
                asm volatile("" : "+v"(i1), "+v"(i2), "+v"(mb));
                const float fs = (float)scale;
                float part = 0.f;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int m = mb + c * T;
                    float y = 0.f;
                    if (m < N) y = fs * ll_cell<MODEL>(rho, m, i1, i2, S1, S2, kc);
                    nv[c] = y;
                    part += y;
                    i1 += rT;
                    i2 += qT;
                    if (i1 >= S1) { i1 -= S1; i2 += 1; }
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int m = tid + c * T;
                    if (m < N) rho[m] = nv[c];
                }
                if (m_renorm > 0 && k % m_renorm == 0 && k < Kmax) {
                    const double tot = ll_block_sum<T>((double)part, scratch);  // includes the barrier
                    scale = tot > 0.0 ? 1.0 / tot : 1.0;  // rho(0) has unit mass
                } else {
                    scale = 1.0;
                    __syncthreads();
                }
            } else {
                __syncthreads();
            }
            if constexpr (JUMP) {  // the observations whose jump count is k
#pragma unroll
                for (int u = 0; u < kLLRecPerThread; ++u) {
                    if (rm[u] < 0 || rt[u] != k) continue;
                    const float v = kHidden ? rho[rm[u]] + rho[rm[u] + hid] : rho[rm[u]];
                    if (!(v > 0.f)) flags |= MJP_FLAG_UNDERFLOW_OBS;
                    else if (v < FLT_MIN) flags |= MJP_FLAG_SUBNORMAL_OBS;
                    a.phi[(int64_t)b * a.n_rec + tid + u * T] = v > 0.f ? log((double)v) : -INFINITY;
                }
                continue;
            }
            // accumulate observed states
#pragma unroll
            for (int u = 0; u < kLLRecPerThread; ++u) {
                if (rm[u] < 0) continue;
                const LLWinL& w = win[rt[u]];
                if (k < w.L || k > w.K) continue;
                const float wt = (k == w.K) ? (float)w.lastw : (float)wbuf[(k & 1) * kLLMaxTimes + rt[u]];
                const float v = kHidden ? rho[rm[u]] + rho[rm[u] + hid] : rho[rm[u]];
                if (k == w.L) {
                    rs[u] = wt * v;
                    rc[u] = 0.f;
                } else {
                    const float yk = fmaf(wt, v, -rc[u]);
                    const float t = rs[u] + yk;
                    rc[u] = (t - rs[u]) - yk;
                    rs[u] = t;
                }
            }
        }
        // log-likelihood: FP64 sum of count * log p over the records
        double tot = 0.0, ninf = 0.0;
        if constexpr (!JUMP) {
            double ll = 0.0;
            bool neg_inf = false;
#pragma unroll
            for (int u = 0; u < kLLRecPerThread; ++u) {
                const int r = tid + u * T;
                if (r >= a.n_rec) continue;
                if (rm[u] < 0) { neg_inf = true; continue; }
                const float p = rs[u] - rc[u];
                if (!(p > 0.f)) {
                    neg_inf = true;
                    flags |= MJP_FLAG_UNDERFLOW_OBS;
                    continue;
                }
                if (p < FLT_MIN) flags |= MJP_FLAG_SUBNORMAL_OBS;
                ll += (double)a.rec[r].count * log((double)p);
            }
            tot = ll_block_sum<T>(ll, scratch);
            ninf = ll_block_sum<T>(neg_inf ? 1.0 : 0.0, scratch);
        }
        if (flags) atomicOr(&flag_sh, flags);
        double mass = 0.0;
        {
            float part = 0.f;
            for (int m = tid; m < N; m += T) part += rho[m];
            mass = ll_block_sum<T>((double)part, scratch);
        }
        if (tid == 0) {
            if (JUMP) {
                if (a.omega_out) a.omega_out[b] = omega;
            } else {
                a.loglik[b] = ninf > 0.0 ? -INFINITY : tot;
            }
            if (a.info) {
                mjp_info inf{};
                inf.omega = omega;
                inf.W = win[a.n_t - 1].W;
                inf.mass_in = x0 >= 0 ? 1.0 : 0.0;
                inf.mass_out = mass;
                inf.K = Kmax;
                inf.L = Lmin;
                inf.flags = (int32_t)flag_sh;
                a.info[b] = inf;
            }
        }
    }
}

// ------------------------------------------------- column kernel (cascade)
//
// The same sweep as k_ll_main for cascade (and birth-death) items, laid out
// so a cell update is a few register operations.  Lane lam = seg * S1 + i1
// of the workgroup owns the cells (i1, seg * len + c), c < len, of one
// column segment and keeps them in registers (C >= len, a template).  In a
// jump its cells are updated in order of c, so the cells above and below
// are the lane's own registers (its old value of cell c - 1 is kept aside),
// except at the segment's two ends, which come from the LDS mirror of the
// whole vector.  Consecutive lanes hold consecutive columns of the same row,
// so the left and right neighbours come from the adjacent lanes by DPP wave
// shifts; lanes 0 and 63 of each wave are ghost lanes that load the two
// columns bordering the wave's 62 real lanes from the mirror and are never
// written back.  Where a segment ends inside a wave (i1 = S1 - 1 next to
// i1 = 0 of the next segment) the rates across the border are zero.
//
// Row m of B: y_m = x_m - (exit terms) x_m + inflows, with each exit rate of
// state m a separate FP32 product (o_b1, o_d1, o_b2, o_d2: the same FP32
// numbers its neighbours pull), so the coefficient of x_m is exactly 1 minus
// the exact sum of the row's off-diagonals and every row of B sums to 1
// exactly; only the rounding of the products and sums remains, which varies
// from jump to jump.
__device__ __forceinline__ float dpp_from_lower_lane(float v) {  // lane l gets lane l - 1 (lane 0: 0)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_upper_lane(float v) {  // lane l gets lane l + 1 (lane 63: 0)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}

template <int MODEL, int C, int CAP>
__global__ __launch_bounds__(kColT) void k_ll_col(LLArgs a, int cls) {
    extern __shared__ char lds[];
    float* rho = reinterpret_cast<float*>(lds);                            // [CAP] the vector's mirror
    double* wbuf = reinterpret_cast<double*>(lds + sizeof(float) * CAP);   // [2][kLLMaxTimes]
    double* scratch = wbuf + 2 * kLLMaxTimes;                              // [16]
    LLWinL* win = reinterpret_cast<LLWinL*>(scratch + 16);                 // [kLLMaxTimes]
    __shared__ int pop_sh[kColT / 64];
    __shared__ unsigned flag_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lam = kColReal * wave + lane - 1;  // column segment of this lane
    const bool ghost = lane == 0 || lane == 63;

    const int first = a.cls_off[cls], last = a.cls_off[cls + 1];
    while (true) {
        const int slot = first + queue_pop(a.queue + cls, pop_sh);
        if (slot >= last) break;
        const int b = a.order[slot];
        const double* th = a.theta + ll_stride(MODEL) * (int64_t)b;
        int S1, S2;
        ll_grid(MODEL, a.dims + 2 * b, S1, S2);
        double w_aw = 0.0;  // the anchor weight of this thread's time (threads tid < n_t)
        if (tid < a.n_t) {
            const LLWin wg = a.win[(int64_t)b * a.n_t + tid];
            win[tid] = ll_win_lds(wg);
            w_aw = wg.aw;
        }
        if (tid == 0) flag_sh = 0u;
        __syncthreads();
        unsigned flags = 0;
        int32_t Kmax = 0, Lmin = INT32_MAX;
        bool over = false;
        for (int j = 0; j < a.n_t; ++j) {
            const int Kj = win[j].K;
            if (Kj < 0) over = true;
            Kmax = max(Kmax, Kj);
            Lmin = min(Lmin, win[j].L);
        }
        const double omega = a.omega_factor * ll_max_exit(MODEL, th, a.dims + 2 * b);
        int cc = 0, nseg = 0, len = 0, S2p = 1;
        const bool fits = col_geom(S1, S2, cc, nseg, len, S2p) && len == C && S1 * S2p <= CAP;
        if (over || !fits) {
            if (tid == 0) {
                a.loglik[b] = -INFINITY;
                if (a.info) {
                    mjp_info inf{};
                    inf.omega = omega;
                    inf.flags = over ? MJP_FLAG_K_LIMIT : MJP_FLAG_OUT_OF_GRID;
                    a.info[b] = inf;
                }
            }
            continue;
        }
        const int NM = S1 * S2p;  // mirror entries
        const int Lam = nseg * S1;
        const double om = omega > 0.0 ? omega : 1.0;
        const float b1 = (float)(th[0] / om), d1 = (float)(th[1] / om);
        const float b2 = MODEL == MJP_MODEL_BD ? 0.f : (float)(th[2] / om);
        const float d2 = MODEL == MJP_MODEL_BD ? 0.f : (float)(th[3] / om);

        // this lane's column segment (ghost lanes: the neighbouring one)
        const bool live = lam >= 0 && lam < Lam;
        const int seg = live ? lam / S1 : 0;
        const int i1 = live ? lam - seg * S1 : 0;
        const int i20 = seg * C;
        const int vl = live ? min(C, S2 - i20) : 0;                 // cells of the lane on the grid
        const bool has_last = live && i20 + C >= S2;                // the grid's last row is cell vl - 1
        const float f1 = (float)i1;
        const float cl = (live && i1 > 0) ? b1 : 0.f;               // inflow from (i1 - 1, i2): k1
        const float cr = (live && i1 + 1 < S1) ? d1 * (f1 + 1.f) : 0.f;  // from (i1 + 1, i2): g1 (i1 + 1)
        const float cu = live ? b2 * f1 : 0.f;                      // from (i1, i2 - 1): k2 i1
        const float ob1 = (live && i1 + 1 < S1) ? b1 : 0.f;         // exits: birth 1 (blocked at the cap),
        const float od1 = live ? d1 * f1 : 0.f;                     //   death 1,
        const float ob2 = cu;                                       //   birth 2 (blocked in the last row)
        float* const col = rho + (live ? i1 * S2p + i20 : 0);       // cell c of the lane at col[c]

        const int x0 = (a.x0_1 < S1 && a.x0_2 < S2) ? a.x0_1 * S2p + a.x0_2 : -1;
        float x[C];
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = (live && c < vl && i1 * S2p + i20 + c == x0) ? 1.f : 0.f;
        for (int m = tid; m < NM; m += kColT) rho[m] = (m == x0) ? 1.f : 0.f;

        // one observation record per thread (the column kernel takes at
        // most kColT records): its mirror index, time, Kahan pair
        int rm = -2, rt = 0;
        float rs = 0.f, rc = 0.f;
        if (tid < a.n_rec) {
            const LLRecord R = a.rec[tid];
            rt = R.t;
            rm = (R.x1 < S1 && R.x2 < S2) ? R.x1 * S2p + R.x2 : -1;
            if (rm < 0) flags |= MJP_FLAG_OUT_OF_GRID;
        }
        if (tid < a.n_t) wbuf[tid] = 0.0;
        __syncthreads();
        if (x0 < 0) flags |= MJP_FLAG_OUT_OF_GRID;

        const int m_renorm = a.renorm_every;
        double wcur = 0.0;  // this time's weight at the current jump (threads tid < n_t)
        for (int k = 0; k <= Kmax; ++k) {
            // weight of jump k for each time (FP64, the recurrence from w_L)
            if (tid < a.n_t) {
                wcur = ll_weight_step(k, win[tid].W, win[tid].L, w_aw, wcur);
                wbuf[(k & 1) * kLLMaxTimes + tid] = wcur;
            }
            if (k > 0) {
                // old values a lane does not hold: ghost columns (rows past
                // the grid read the mirror's zeros), segment ends
                if (ghost) {
#pragma unroll
                    for (int c = 0; c < C; ++c) x[c] = live ? col[c] : 0.f;
                }
                const float up = (live && i20 > 0) ? col[-1] : 0.f;
                const float dn = (live && i20 + C < S2) ? col[C] : 0.f;
                __syncthreads();  // every read of the old vector is done
                float xu = up;
                float fp = (float)i20;   // f2 of cell c
                float p = d2 * fp;       // its exit by death 2: g2 i2
                int rem = vl;            // cells of the lane from c on
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    // per-cell tests from a loop-carried counter the compiler
                    // cannot precompute for all c (that would hold C masks live)
                    asm volatile("" : "+v"(rem));
                    // the cell below: the lane's next cell, or past the
                    // segment's end the next segment's first (0 off the grid)
                    const float xd = (c + 1 < C) ? ((rem == 1) ? dn : x[c + 1]) : dn;
                    const float xc = x[c];
                    const float xl = dpp_from_lower_lane(xc);
                    const float xr = dpp_from_upper_lane(xc);
                    const float fp1 = fp + 1.f;
                    const float cd = d2 * fp1;            // inflow from (i1, i2 + 1): g2 (i2 + 1)
                    const float q = (has_last && rem == 1) ? 0.f : ob2;
                    float acc = cl * xl;
                    acc = fmaf(cr, xr, acc);
                    acc = fmaf(cu, xu, acc);
                    acc = fmaf(cd, xd, acc);
                    acc = fmaf(-q, xc, acc);
                    acc = fmaf(-p, xc, acc);
                    acc = fmaf(-od1, xc, acc);
                    acc = fmaf(-ob1, xc, acc);
                    const float y = xc + acc;
                    xu = xc;
                    x[c] = rem > 0 ? y : 0.f;  // rows past the grid stay 0
                    p = cd;
                    fp = fp1;
                    rem -= 1;
                }
                if (m_renorm > 0 && k % m_renorm == 0 && k < Kmax) {
                    float part = 0.f;
                    if (!ghost) {
#pragma unroll
                        for (int c = 0; c < C; ++c) part += x[c];  // cells past len and off the grid hold 0
                    }
                    const double tot = ll_block_sum<kColT>((double)part, scratch);
                    const float fs = tot > 0.0 ? (float)(1.0 / tot) : 1.f;  // rho(0) has unit mass
#pragma unroll
                    for (int c = 0; c < C; ++c) x[c] *= fs;
                }
                if (!ghost && live) {
#pragma unroll
                    for (int c = 0; c < C; ++c) col[c] = x[c];  // rows past the grid write their zeros
                }
                __syncthreads();
            } else {
                __syncthreads();
            }
            if (rm >= 0) {
                const LLWinL& w = win[rt];
                if (k >= w.L && k <= w.K) {
                    const float wt = (k == w.K) ? (float)w.lastw : (float)wbuf[(k & 1) * kLLMaxTimes + rt];
                    const float v = rho[rm];
                    if (k == w.L) {
                        rs = wt * v;
                        rc = 0.f;
                    } else {
                        const float yk = fmaf(wt, v, -rc);
                        const float t = rs + yk;
                        rc = (t - rs) - yk;
                        rs = t;
                    }
                }
            }
        }
        double ll = 0.0;
        bool neg_inf = false;
        if (tid < a.n_rec) {
            const float pr = rs - rc;
            if (rm < 0) {
                neg_inf = true;
            } else if (!(pr > 0.f)) {
                neg_inf = true;
                flags |= MJP_FLAG_UNDERFLOW_OBS;
            } else {
                if (pr < FLT_MIN) flags |= MJP_FLAG_SUBNORMAL_OBS;
                ll = (double)a.rec[tid].count * log((double)pr);
            }
        }
        const double tot = ll_block_sum<kColT>(ll, scratch);
        const double ninf = ll_block_sum<kColT>(neg_inf ? 1.0 : 0.0, scratch);
        if (flags) atomicOr(&flag_sh, flags);
        float part = 0.f;
        for (int m = tid; m < NM; m += kColT) part += rho[m];
        const double mass = ll_block_sum<kColT>((double)part, scratch);
        if (tid == 0) {
            a.loglik[b] = ninf > 0.0 ? -INFINITY : tot;
            if (a.info) {
                mjp_info inf{};
                inf.omega = omega;
                inf.W = win[a.n_t - 1].W;
                inf.mass_in = x0 >= 0 ? 1.0 : 0.0;
                inf.mass_out = mass;
                inf.K = Kmax;
                inf.L = Lmin;
                inf.flags = (int32_t)flag_sh;
                a.info[b] = inf;
            }
        }
    }
}

// ------------------------------------------------------- cluster kernel
//
// The cell kernel's sweep (k_ll_main: the same weights, renormalisation and
// record accumulation; the column kernel's cell update) for an item too large for one
// workgroup's LDS, run by a cluster of kClG workgroups of one cooperative
// launch.  Cluster c takes the items c, c + nclust, ... of the class (cost
// order), so every workgroup of a cluster knows the item without a
// broadcast.  Workgroup r of a cluster owns the states [lo, hi) =
// [r len, (r + 1) len), len = ceil(N / kClG), and keeps them in LDS with a
// halo of SJ reaches on each side (reach = S1 states, the pull rows'
// farthest column; SJ = kClJumps where the item allows, else 1).  A round
// is SJ jumps; jump j of a round updates the own states and the halo states
// still (SJ - j) reaches deep (the same cell update the halo's owner makes,
// so the same bits): the new values into registers, a barrier, into LDS.
// At a round's end the SJ reach states at each end of the own range go to
// the cluster's exchange buffer (device-scope stores, the slot of the
// round's parity); every wave drains its stores; the workgroup publishes the
// number of rounds done on its flag and waits for its neighbours' (all of
// the cluster's at a renormalisation, which falls on a round's end and whose
// block sums travel the same way); it then reads its halo from the
// neighbours' slots (device-scope loads).  Every
// wait has the 2 s deadline of the persistent sweeps: on a miss the abort
// word is raised and every workgroup leaves, the items not finished keep
// the NaN k_ll_order wrote.  At the end of an item each workgroup's FP64 sum
// of count log p over the records of its own states meets the others' in
// the same way and rank 0 adds them in rank order.
struct ClArgs {
    LLArgs a;
    float* __restrict__ xbuf;      // [nclust][2][kClG][2][kClSlot] boundary states
    double* __restrict__ part;     // [nclust][4][kClG] block sums: renormalisation masses (two
                                   // slots, alternating), an item's log-lik and mass
    double* __restrict__ ninf;     // [nclust][2][kClG] count of records with no probability; flags (as a double)
    unsigned* __restrict__ wflag;  // [nclust][kClG][32] jumps (exchange rounds) done
    unsigned* __restrict__ abort_word;
    uint64_t timeout_ticks;
    int32_t nclust;
};

// The column kernel's cell update for the cluster kernel's models (birth-
// death and cascade), neighbours read from LDS: y = x + (inflows - exits x)
// with each exit rate a separate FP32 product (the numbers its neighbours
// pull), no FP64 diagonal.
template <int MODEL>
__device__ __forceinline__ float cl_cell(const float* rho, int m, int i1, int i2, int S1, int S2, const LLCoef& k) {
    static_assert(MODEL == MJP_MODEL_BD || MODEL == MJP_MODEL_CASCADE2, "birth-death and cascade only");
    const float b1 = k.c[0], d1 = k.c[1], b2 = k.c[2], d2 = k.c[3];
    const float f1 = (float)i1, f2 = (float)i2;
    const bool left = i1 > 0, right = i1 + 1 < S1, up = i2 > 0, down = i2 + 1 < S2;
    const float xc = rho[m];
    const float xl = left ? rho[m - 1] : 0.f;
    const float xr = right ? rho[m + 1] : 0.f;
    const float xu = up ? rho[m - S1] : 0.f;
    const float xd = down ? rho[m + S1] : 0.f;
    const float cl = left ? b1 : 0.f;                 // inflow from (i1 - 1, i2): k1
    const float cr = right ? d1 * (f1 + 1.f) : 0.f;   // from (i1 + 1, i2): g1 (i1 + 1)
    const float cu = b2 * f1;                         // from (i1, i2 - 1): k2 i1
    const float cd = d2 * (f2 + 1.f);                 // from (i1, i2 + 1): g2 (i2 + 1)
    const float q = down ? cu : 0.f;                  // exits: birth 2 (blocked in the last row),
    const float p = d2 * f2;                          //   death 2,
    const float od1 = d1 * f1;                        //   death 1,
    const float ob1 = right ? b1 : 0.f;               //   birth 1 (blocked at the cap)
    float acc = cl * xl;
    acc = fmaf(cr, xr, acc);
    acc = fmaf(cu, xu, acc);
    acc = fmaf(cd, xd, acc);
    acc = fmaf(-q, xc, acc);
    acc = fmaf(-p, xc, acc);
    acc = fmaf(-od1, xc, acc);
    acc = fmaf(-ob1, xc, acc);
    return xc + acc;
}

// Publish `round` on my flag and wait until the workgroups of my cluster in
// [rlo, rhi] have published it (bounded); false if the sweep aborted.
__device__ __forceinline__ bool cl_sync(unsigned* wf, int r, int rlo, int rhi, unsigned round, unsigned* abort_word,
                                        uint64_t timeout_ticks) {
    __shared__ int aborted;
    drain_wave<true>();
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane == 0) {
            aborted = 0;
            __hip_atomic_store(&wf[r * 32], round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const int h = rlo + lane;
        bool bad = false;
        if (h <= rhi && h != r) {
            const uint64_t t0 = wall_clock64();
            unsigned spins = 0;
            while (__hip_atomic_load(&wf[h * 32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < round) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins % kAbortCheckEvery != 0) continue;
                if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    bad = true;
                    break;
                }
                if (wall_clock64() - t0 > timeout_ticks) {
                    __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bad = true;
                    break;
                }
            }
        }
        if (bad) aborted = 1;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(aborted) == 0;  // uniform: every thread read the same word
}

template <int MODEL>
__global__ __launch_bounds__(kClT) void k_ll_cluster(ClArgs ca) {
    constexpr int T = kClT, C = kClC;
    constexpr int CAP = kClOwn + 2 * kClSlot;  // own states and both halos
    const LLArgs& a = ca.a;
    extern __shared__ __align__(16) char lds[];
    float* lx = reinterpret_cast<float*>(lds);                             // [CAP]
    double* wbuf = reinterpret_cast<double*>(lds + sizeof(float) * CAP);   // [2][kLLMaxTimes]
    double* scratch = wbuf + 2 * kLLMaxTimes;                              // [16]
    LLWinL* win = reinterpret_cast<LLWinL*>(scratch + 16);                 // [kLLMaxTimes]
    __shared__ unsigned flag_sh;
    const int tid = threadIdx.x;
    const int cl = blockIdx.x / kClG, r = blockIdx.x - cl * kClG;
    const int first = a.cls_off[kClClass], last = a.cls_off[kClClass + 1];
    unsigned* wf = ca.wflag + (size_t)cl * kClG * 32;
    float* xb = ca.xbuf + (size_t)cl * 2 * kClG * 2 * kClSlot;
    double* pt = ca.part + (size_t)cl * 4 * kClG;
    unsigned round = 0;  // exchange rounds done (the same in every workgroup of the cluster)
    for (int slot = first + cl; slot < last; slot += ca.nclust) {
        const int b = a.order[slot];
        const double* th = a.theta + ll_stride(MODEL) * (int64_t)b;
        int S1, S2;
        ll_grid(MODEL, a.dims + 2 * b, S1, S2);
        double w_aw = 0.0;  // the anchor weight of this thread's time (threads tid < n_t)
        if (tid < a.n_t) {
            const LLWin wg = a.win[(int64_t)b * a.n_t + tid];
            win[tid] = ll_win_lds(wg);
            w_aw = wg.aw;
        }
        if (tid == 0) flag_sh = 0u;
        __syncthreads();
        unsigned flags = 0;
        int32_t Kmax = 0, Lmin = INT32_MAX;
        bool over = false;
        for (int j = 0; j < a.n_t; ++j) {
            const int Kj = win[j].K;
            if (Kj < 0) over = true;
            Kmax = max(Kmax, Kj);
            Lmin = min(Lmin, win[j].L);
        }
        const int64_t N64 = (int64_t)S1 * S2;
        const double omega = a.omega_factor * ll_max_exit(MODEL, th, a.dims + 2 * b);
        const int reach = MODEL == MJP_MODEL_BD ? 1 : S1;
        if (over || S1 < 1 || S2 < 1 || N64 > kClMaxStates || reach > kClReachMax) {
            if (r == 0 && tid == 0) {
                a.loglik[b] = -INFINITY;
                if (a.info) {
                    mjp_info inf{};
                    inf.omega = omega;
                    inf.flags = over ? MJP_FLAG_K_LIMIT : MJP_FLAG_OUT_OF_GRID;
                    a.info[b] = inf;
                }
            }
            continue;
        }
        const int N = (int)N64;
        const int len = (N + kClG - 1) / kClG;
        const int lo = min(N, r * len), hi = min(N, lo + len);
        // jumps per exchange: kClJumps where the renormalisation points end a
        // round, the deeper halo fits its slot and LDS, and every jump's
        // cells fit the threads' registers (unless the caller asked for one);
        // else one
        const int SJ = (!a.one_jump && a.renorm_every % kClJumps == 0 && kClJumps * reach <= kClSlot &&
                        len >= kClJumps * reach && len + 2 * (kClJumps - 1) * reach <= kClOwn)
                           ? kClJumps
                           : 1;
        const int ext = SJ * reach;  // halo depth
        const int hlo = max(0, lo - ext), hhi = min(N, hi + ext);
        float* rho = lx - hlo;  // rho[m] for m in [hlo, hhi)
        const double om = omega > 0.0 ? omega : 1.0;
        LLCoef kc;
#pragma unroll
        for (int i = 0; i < 6; ++i) kc.c[i] = i < ll_params(MODEL) ? (float)(th[i] / om) : 0.f;
        kc.NP = 1;
        const int x0lim2 = S2;
        const int x0 = (a.x0_1 < S1 && a.x0_2 < x0lim2) ? a.x0_1 + S1 * a.x0_2 : -1;
        for (int m = hlo + tid; m < hhi; m += T) rho[m] = (m == x0) ? 1.f : 0.f;

        // the records whose state this workgroup owns
        int rm[kLLRecPerThread], rt[kLLRecPerThread];
        float rs[kLLRecPerThread], rc[kLLRecPerThread];
        bool any_off = false;
#pragma unroll
        for (int u = 0; u < kLLRecPerThread; ++u) {
            const int rr = tid + u * T;
            rm[u] = -2;
            rt[u] = 0;
            rs[u] = 0.f;
            rc[u] = 0.f;
            if (rr < a.n_rec) {
                const LLRecord R = a.rec[rr];
                const int m = (R.x1 < S1 && R.x2 < S2) ? R.x1 + S1 * R.x2 : -1;
                if (m < 0) {
                    any_off = true;  // every workgroup sees it; rank 0 reports it
                } else if (m >= lo && m < hi) {
                    rm[u] = m;
                    rt[u] = R.t;
                }
            }
        }
        if (any_off && r == 0) flags |= MJP_FLAG_OUT_OF_GRID;
        if (tid < a.n_t) wbuf[tid] = 0.0;
        __syncthreads();
        if (x0 < 0 && r == 0) flags |= MJP_FLAG_OUT_OF_GRID;

        const int qT = T / S1, rT = T - qT * S1;
        double scale = 1.0;
        const int m_renorm = a.renorm_every;
        int rpar = 0;
        double wcur = 0.0;  // this time's weight at the current jump (threads tid < n_t)
        const __amdgpu_buffer_rsrc_t xr = iter_rsrc(xb, (int64_t)2 * kClG * 2 * kClSlot);
        bool ok = true;
        for (int k = 0; k <= Kmax && ok; ++k) {
            // weight of jump k for each time (FP64, the recurrence from w_L)
            if (tid < a.n_t) {
                wcur = ll_weight_step(k, win[tid].W, win[tid].L, w_aw, wcur);
                wbuf[(k & 1) * kLLMaxTimes + tid] = wcur;
            }
            if (k > 0) {
                // jump j of its round: the own states and the halo states still
                // (SJ - j) reaches deep, from values one reach deeper (the
                // same cell update the halo's owner makes, so the same bits)
                const int j = (k - 1) % SJ + 1;
                const int e = (SJ - j) * reach;
                const int clo = max(0, lo - e), chi = min(N, hi + e);
                const int s0 = clo + tid;
                float nv[C];
                int i1 = s0 % S1, i2 = s0 / S1, mb = s0;
                asm volatile("" : "+v"(i1), "+v"(i2), "+v"(mb));
                const float fs = (float)scale;
                scale = 1.0;
                float part = 0.f;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int m = mb + c * T;
                    float y = 0.f;
                    if (m < chi) y = fs * cl_cell<MODEL>(rho, m, i1, i2, S1, S2, kc);
                    nv[c] = y;
                    if (m >= lo && m < hi) part += y;
                    i1 += rT;
                    i2 += qT;
                    if (i1 >= S1) { i1 -= S1; i2 += 1; }
                }
                __syncthreads();  // every read of the old values is done
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int m = s0 + c * T;
                    if (m < chi) rho[m] = nv[c];
                }
                if (j == SJ) {
                    // round end: the first and last ext own states into this
                    // round's slot ([parity][r][0], [parity][r][1])
                    const uint32_t sbase = (uint32_t)(((((k / SJ) & 1) * kClG + r) * 2) * kClSlot);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const int m = s0 + c * T;
                        if (m >= lo && m < hi) {
                            if (m - lo < ext) st_iter<true>(xr, 4u * (sbase + (uint32_t)(m - lo)), nv[c]);
                            if (hi - m <= ext)
                                st_iter<true>(xr, 4u * (sbase + kClSlot + (uint32_t)(m - (hi - ext))), nv[c]);
                        }
                    }
                    const bool renorm = m_renorm > 0 && k % m_renorm == 0 && k < Kmax;
                    if (renorm) {
                        const double s = ll_block_sum<T>((double)part, scratch);
                        if (tid == 0)
                            __hip_atomic_store(pt + rpar * kClG + r, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    ++round;
                    ok = renorm ? cl_sync(wf, r, 0, kClG - 1, round, ca.abort_word, ca.timeout_ticks)
                                : cl_sync(wf, r, max(0, r - 1), min(kClG - 1, r + 1), round, ca.abort_word,
                                          ca.timeout_ticks);
                    if (!ok) break;
                    // the halo from the neighbours' slots of this round
                    const uint32_t pb = (uint32_t)(((k / SJ) & 1) * kClG);
                    for (int m = hlo + tid; m < lo; m += T) {  // rank r - 1's last ext states
                        const uint32_t o = (uint32_t)(((pb + (r - 1)) * 2 + 1) * kClSlot) + (uint32_t)(m - (lo - ext));
                        rho[m] = ld_iter<true>(xr, 4u * o);
                    }
                    for (int m = hi + tid; m < hhi; m += T) {  // rank r + 1's first ext states
                        const uint32_t o = (uint32_t)(((pb + (r + 1)) * 2) * kClSlot) + (uint32_t)(m - hi);
                        rho[m] = ld_iter<true>(xr, 4u * o);
                    }
                    if (renorm) {
                        double tot = 0.0;
                        for (int q = 0; q < kClG; ++q)
                            tot += __hip_atomic_load(pt + rpar * kClG + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        scale = tot > 0.0 ? 1.0 / tot : 1.0;  // rho(0) has unit mass
                        rpar ^= 1;
                    }
                }
                __syncthreads();
            } else {
                __syncthreads();
            }
#pragma unroll
            for (int u = 0; u < kLLRecPerThread; ++u) {
                if (rm[u] < 0) continue;
                const LLWinL& w = win[rt[u]];
                if (k < w.L || k > w.K) continue;
                const float wt = (k == w.K) ? (float)w.lastw : (float)wbuf[(k & 1) * kLLMaxTimes + rt[u]];
                const float v = rho[rm[u]];
                if (k == w.L) {
                    rs[u] = wt * v;
                    rc[u] = 0.f;
                } else {
                    const float yk = fmaf(wt, v, -rc[u]);
                    const float t = rs[u] + yk;
                    rc[u] = (t - rs[u]) - yk;
                    rs[u] = t;
                }
            }
        }
        if (!ok) return;  // aborted: every workgroup leaves
        double ll = 0.0, nneg = 0.0;
#pragma unroll
        for (int u = 0; u < kLLRecPerThread; ++u) {
            if (rm[u] < 0) continue;
            const float p = rs[u] - rc[u];
            if (!(p > 0.f)) {
                nneg += 1.0;
                flags |= MJP_FLAG_UNDERFLOW_OBS;
                continue;
            }
            if (p < FLT_MIN) flags |= MJP_FLAG_SUBNORMAL_OBS;
            ll += (double)a.rec[tid + u * T].count * log((double)p);
        }
        const double tot = ll_block_sum<T>(ll, scratch);
        const double bad = ll_block_sum<T>(nneg, scratch);
        float mpart = 0.f;
        for (int m = lo + tid; m < hi; m += T) mpart += rho[m];
        const double mass = ll_block_sum<T>((double)mpart, scratch);
        if (flags) atomicOr(&flag_sh, flags);
        __syncthreads();
        // the workgroups' sums meet in slots of their own (a workgroup that
        // is not my neighbour may still read the renormalisation slots)
        if (tid == 0) {
            __hip_atomic_store(pt + 2 * kClG + r, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(pt + 3 * kClG + r, mass, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ca.ninf + (size_t)cl * 2 * kClG + r, bad + (double)(flag_sh & MJP_FLAG_OUT_OF_GRID ? 1 : 0),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ca.ninf + (size_t)cl * 2 * kClG + kClG + r, (double)flag_sh, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        ++round;
        if (!cl_sync(wf, r, 0, kClG - 1, round, ca.abort_word, ca.timeout_ticks)) return;
        if (r == 0 && tid == 0) {
            double sll = 0.0, smass = 0.0, sbad = 0.0;
            unsigned sflags = 0u;
            for (int q = 0; q < kClG; ++q) {
                sll += __hip_atomic_load(pt + 2 * kClG + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                smass += __hip_atomic_load(pt + 3 * kClG + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sbad += __hip_atomic_load(ca.ninf + (size_t)cl * 2 * kClG + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sflags |= (unsigned)__hip_atomic_load(ca.ninf + (size_t)cl * 2 * kClG + kClG + q, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            }
            a.loglik[b] = sbad > 0.0 ? -INFINITY : sll;
            if (a.info) {
                mjp_info inf{};
                inf.omega = omega;
                inf.W = win[a.n_t - 1].W;
                inf.mass_in = x0 >= 0 ? 1.0 : 0.0;
                inf.mass_out = smass;
                inf.K = Kmax;
                inf.L = Lmin;
                inf.flags = (int32_t)sflags;  // every workgroup's flags
                a.info[b] = inf;
            }
        }
        // the end-of-item slots are reused by the next item only after
        // another cluster-wide round: nobody overwrites them before rank 0
        // read them (and the renormalisation slots of this item are free)
        ++round;
        if (!cl_sync(wf, r, 0, kClG - 1, round, ca.abort_word, ca.timeout_ticks)) return;
    }
}

__global__ void k_ll_zero_u32(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- host

using MainFn = void (*)(LLArgs, int);

template <int MODEL, size_t... S>
constexpr std::array<MainFn, kLLNumShapes> ll_row(std::index_sequence<S...>) {
    return {{&k_ll_main<MODEL, kLLShapes[S].T, kLLShapes[S].C>...}};
}
// kernel of (model, shape)
static const std::array<MainFn, kLLNumShapes> kLLMains[4] = {
    ll_row<MJP_MODEL_BD>(std::make_index_sequence<kLLNumShapes>{}),
    ll_row<MJP_MODEL_CASCADE2>(std::make_index_sequence<kLLNumShapes>{}),
    ll_row<MJP_MODEL_TWOSTATE>(std::make_index_sequence<kLLNumShapes>{}),
    ll_row<MJP_MODEL_AUTOREG>(std::make_index_sequence<kLLNumShapes>{})};

// jump-mode kernels of (model, class): the default shape of each class
template <int MODEL, size_t... S>
constexpr std::array<MainFn, kLLClasses> jp_row(std::index_sequence<S...>) {
    return {{&k_ll_main<MODEL, kLLShapes[kLLDefaultShape[S]].T, kLLShapes[kLLDefaultShape[S]].C, true>...}};
}
static const std::array<MainFn, kLLClasses> kJpMains[4] = {
    jp_row<MJP_MODEL_BD>(std::make_index_sequence<kLLClasses>{}),
    jp_row<MJP_MODEL_CASCADE2>(std::make_index_sequence<kLLClasses>{}),
    jp_row<MJP_MODEL_TWOSTATE>(std::make_index_sequence<kLLClasses>{}),
    jp_row<MJP_MODEL_AUTOREG>(std::make_index_sequence<kLLClasses>{})};

// column kernels of (model BD / cascade, column class)
template <int MODEL, size_t... S>
constexpr std::array<MainFn, kColClasses> col_row(std::index_sequence<S...>) {
    return {{&k_ll_col<MODEL, kColCs[S], col_cap(S)>...}};
}
static const std::array<MainFn, kColClasses> kColMains =
    col_row<MJP_MODEL_CASCADE2>(std::make_index_sequence<kColClasses>{});
// LDS after the column kernel's mirror: weights [2][kLLMaxTimes], block-sum
// scratch [16] (FP64), windows [kLLMaxTimes]; with the mirror at most
// kColMirror floats the block stays within one CU's 160 KB
constexpr size_t kColExtra = sizeof(double) * (2 * kLLMaxTimes + 16) + sizeof(LLWinL) * kLLMaxTimes;
static_assert(sizeof(float) * kColMirror + kColExtra + 64 <= 160 * 1024, "column kernel LDS exceeds a CU");
inline size_t col_lds(int cc) { return sizeof(float) * (size_t)col_cap(cc) + kColExtra; }
inline bool col_model(int model) { return model == MJP_MODEL_CASCADE2; }
// LDS of a cluster workgroup: own states and halos, then the weights,
// block-sum scratch and windows (as the column kernel's extras)
inline size_t cl_lds() { return sizeof(float) * (size_t)(kClOwn + 2 * kClSlot) + kColExtra; }

inline size_t ll_lds(int shape) {
    return sizeof(float) * (size_t)ll_cap(kLLShapes[shape].T, kLLShapes[shape].C) + kLLExtraLds;
}
// a shape may run class c with n_rec records if it holds the class's largest
// item and has a record slot per record
inline bool ll_eligible(int shape, int cls, int n_rec) {
    return ll_cap(kLLShapes[shape].T, kLLShapes[shape].C) >= kLLClassCap[cls] &&
           n_rec <= kLLRecPerThread * kLLShapes[shape].T;
}

// ---------------------------------------------------------------- host state
//
// Per device, kept until the process ends:
//  * kernel attributes, occupancies and the chosen shape per (model, class);
//  * every observation set seen so far, in its own device buffers, written
//    once by a copy on the stream of the first call that used it and never
//    rewritten: work already enqueued, and a graph captured from a call, keep
//    reading the records they were enqueued with;
//  * the work tables (windows, costs, order, queue counters, class offsets)
//    per stream, so calls on different streams never share them.
constexpr int kLLMaxObsSets = 256;  // kept per device; the least recently used is freed beyond that
constexpr int kLLMaxStreams = 64;   // work tables per device; likewise
constexpr int kLLMaxDevices = 64;

static_assert(sizeof(LLRecord) == 4 * sizeof(int32_t), "records are the caller's (t, x1, x2, count) rows");

struct LLObsSet {
    std::vector<LLRecord> rec;
    std::vector<double> T;
    DevBuf rec_d, T_d;
};

// A call's size classes are launched round-robin on the caller's stream and
// kLLAux streams forked from it (and joined back before the call returns),
// so the tail of one class -- a few long items while most CUs idle -- runs
// beside the next class's items.  Each caller stream has its own forked
// streams (default priority), so a graph captured on one stream forks and
// joins only its own.
constexpr int kLLAux = 3;

struct LLWork {
    hipStream_t stream = nullptr;
    DevBuf win, cost, order, queue, cls_off;
    DevBuf cl_x, cl_part, cl_ninf, cl_flag;  // clusters: exchange slots, sums, flags + abort word
    hipStream_t aux[kLLAux] = {};
    hipEvent_t fork = nullptr, join[kLLAux] = {};
    void release() {
        for (DevBuf* d : {&win, &cost, &order, &queue, &cls_off, &cl_x, &cl_part, &cl_ninf, &cl_flag}) d->release();
        for (int i = 0; i < kLLAux; ++i) {
            if (aux[i]) (void)hipStreamDestroy(aux[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
            aux[i] = nullptr;
            join[i] = nullptr;
        }
        if (fork) (void)hipEventDestroy(fork);
        fork = nullptr;
    }
};

// Device tables of one call.
struct LLBufs {
    const LLRecord* rec = nullptr;
    const double* T = nullptr;
    LLWin* win = nullptr;
    float* cost = nullptr;
    int32_t* order = nullptr;
    unsigned* queue = nullptr;
    int32_t* cls_off = nullptr;
    float* cl_x = nullptr;  // null: no clusters (items above kLLMaxStates get -inf)
    double* cl_part = nullptr;
    double* cl_ninf = nullptr;
    unsigned* cl_flag = nullptr;
};

struct LLContext {
    std::mutex mu;
    int device = -1, ncu = 0;
    std::vector<std::unique_ptr<LLObsSet>> obs;  // most recently used first
    std::vector<std::unique_ptr<LLWork>> work;
    bool attr_set = false;
    int occ[4][kLLNumShapes] = {};  // resident workgroups per CU (0 = not queried)
    int occ_jp[4][kLLClasses] = {};  // the same for the jump-mode kernels
    int occ_col[kColClasses] = {};  // the same for the column kernels (cascade)
    int nclust = 0;                 // clusters of the cluster kernel that fit co-resident (0: none)
    int cl_occ = 0, cl_coop = 0;    // its workgroups per CU, cooperative launch support
    int wall_khz = 0;
    int shape[4][kLLClasses];       // chosen shape per (model, class); -1 = default
    int kernel[4] = {MJP_LL_KERNEL_AUTO, MJP_LL_KERNEL_AUTO, MJP_LL_KERNEL_AUTO, MJP_LL_KERNEL_AUTO};
    LLContext() {
        for (auto& m : shape)
            for (int& c : m) c = -1;
    }
};

static LLContext* ll_contexts() {
    static LLContext ctxs[kLLMaxDevices];
    return ctxs;
}
static LLContext& ctx_for(int dev) { return ll_contexts()[dev]; }

// Frees every device table the log-likelihood calls keep (observation sets,
// per-stream work tables) on every device; the next call rebuilds them.
mjp_status ll_release_all() {
    for (int dev = 0; dev < kLLMaxDevices; ++dev) {
        LLContext& C = ll_contexts()[dev];
        std::lock_guard<std::mutex> lock(C.mu);
        if (C.obs.empty() && C.work.empty()) continue;
        MJP_HIP(hipSetDevice(dev));
        MJP_HIP(hipDeviceSynchronize());
        for (auto& o : C.obs) {
            o->rec_d.release();
            o->T_d.release();
        }
        for (auto& w : C.work) w->release();
        C.obs.clear();
        C.work.clear();
    }
    return MJP_OK;
}

}  // namespace mjp

using namespace mjp;

namespace mjp {

// kernel attributes and occupancies, once per device
static mjp_status ll_attrs(LLContext& C, int dev) {
    if (C.attr_set) return MJP_OK;
    for (int m = 0; m < 4; ++m)
        for (int sid = 0; sid < kLLNumShapes; ++sid) {
            MJP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kLLMains[m][sid]),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)ll_lds(sid)));
            int nb = 0;
            MJP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kLLMains[m][sid], kLLShapes[sid].T, ll_lds(sid)));
            C.occ[m][sid] = std::max(nb, 1);
        }
    for (int m = 0; m < 4; ++m)
        for (int c = 0; c < kLLClasses; ++c) {
            const int sid = kLLDefaultShape[c];
            MJP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kJpMains[m][c]),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)ll_lds(sid)));
            int nb = 0;
            MJP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kJpMains[m][c], kLLShapes[sid].T, ll_lds(sid)));
            C.occ_jp[m][c] = std::max(nb, 1);
        }
    for (int cc = 0; kColEnabled && cc < kColClasses; ++cc) {
        MJP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kColMains[cc]),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)col_lds(cc)));
        int nb = 0;
        MJP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kColMains[cc], kColT, col_lds(cc)));
        C.occ_col[cc] = std::max(nb, 1);
    }
    MJP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_ll_order), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(unsigned long long) * kLLMaxSort)));
    MJP_HIP(hipDeviceGetAttribute(&C.ncu, hipDeviceAttributeMultiprocessorCount, dev));
    {  // clusters: one cooperative launch, every workgroup co-resident
        int coop = 0, occ = 0;
        MJP_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        // the wall-clock rate of the wait deadlines (100 MHz where not reported, as
        // in the persistent sweep)
        if (hipDeviceGetAttribute(&C.wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || C.wall_khz <= 0) {
            (void)hipGetLastError();
            C.wall_khz = 100000;
        }
        for (const void* f : {reinterpret_cast<const void*>(k_ll_cluster<MJP_MODEL_BD>),
                              reinterpret_cast<const void*>(k_ll_cluster<MJP_MODEL_CASCADE2>)}) {
            MJP_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cl_lds()));
            int nb = 0;
            MJP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kClT, cl_lds()));
            occ = occ == 0 ? nb : std::min(occ, nb);
        }
        C.cl_occ = occ;
        C.cl_coop = coop;
        C.nclust = (coop && occ >= 1) ? C.ncu * occ / kClG : 0;
    }
    C.device = dev;
    C.attr_set = true;
    return MJP_OK;
}

// The device copy of an observation set: found among the sets seen before,
// or uploaded once with a copy on stream s (from host vectors the set keeps).
static mjp_status ll_obs(LLContext& C, const std::vector<LLRecord>& recs, const mjp_obs* obs, hipStream_t s,
                         LLBufs& bf) {
    const size_t nrec = recs.size(), nt = (size_t)obs->n_t;
    for (size_t i = 0; i < C.obs.size(); ++i) {
        LLObsSet& o = *C.obs[i];
        if (o.rec.size() != nrec || o.T.size() != nt) continue;
        if (nrec && std::memcmp(o.rec.data(), recs.data(), sizeof(LLRecord) * nrec) != 0) continue;
        if (std::memcmp(o.T.data(), obs->T_h, sizeof(double) * nt) != 0) continue;
        if (i > 0) std::rotate(C.obs.begin(), C.obs.begin() + i, C.obs.begin() + i + 1);
        bf.rec = C.obs[0]->rec_d.as<LLRecord>();
        bf.T = C.obs[0]->T_d.as<double>();
        return MJP_OK;
    }
    if ((int)C.obs.size() >= kLLMaxObsSets) {  // free the least recently used set once nothing reads it
        MJP_HIP(hipDeviceSynchronize());
        C.obs.back()->rec_d.release();
        C.obs.back()->T_d.release();
        C.obs.pop_back();
    }
    std::unique_ptr<LLObsSet> o(new (std::nothrow) LLObsSet());
    MJP_CHECK(o, MJP_E_DEVICE, "out of host memory");
    o->rec = recs;
    o->T.assign(obs->T_h, obs->T_h + nt);
    mjp_status st;
    if ((st = o->rec_d.reserve(sizeof(LLRecord) * std::max<size_t>(nrec, 1))) ||
        (st = o->T_d.reserve(sizeof(double) * nt)))
        return st;
    if (nrec) MJP_HIP(hipMemcpyAsync(o->rec_d.ptr, o->rec.data(), sizeof(LLRecord) * nrec, hipMemcpyHostToDevice, s));
    MJP_HIP(hipMemcpyAsync(o->T_d.ptr, o->T.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));
    bf.rec = o->rec_d.as<LLRecord>();
    bf.T = o->T_d.as<double>();
    C.obs.insert(C.obs.begin(), std::move(o));
    return MJP_OK;
}

// The work tables of stream s, grown to B items of n_t times.
static mjp_status ll_work(LLContext& C, hipStream_t s, int B, int n_t, LLBufs& bf, LLWork** wout = nullptr) {
    LLWork* w = nullptr;
    for (size_t i = 0; i < C.work.size(); ++i)  // most recently used first
        if (C.work[i]->stream == s) {
            if (i > 0) std::rotate(C.work.begin(), C.work.begin() + i, C.work.begin() + i + 1);
            w = C.work[0].get();
            break;
        }
    if (!w) {
        if ((int)C.work.size() >= kLLMaxStreams) {  // free the least recently used stream's tables
            MJP_HIP(hipDeviceSynchronize());
            C.work.back()->release();
            C.work.pop_back();
        }
        std::unique_ptr<LLWork> nw(new (std::nothrow) LLWork());
        MJP_CHECK(nw, MJP_E_DEVICE, "out of host memory");
        nw->stream = s;
        for (int i = 0; i < kLLAux; ++i) {
            if (hipStreamCreateWithFlags(&nw->aux[i], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&nw->join[i], hipEventDisableTiming) != hipSuccess) {
                nw->release();
                return fail(MJP_E_DEVICE, "could not create the forked streams of a likelihood call");
            }
        }
        if (hipEventCreateWithFlags(&nw->fork, hipEventDisableTiming) != hipSuccess) {
            nw->release();
            return fail(MJP_E_DEVICE, "could not create the forked streams of a likelihood call");
        }
        C.work.insert(C.work.begin(), std::move(nw));
        w = C.work[0].get();
    }
    if (wout) *wout = w;
    mjp_status st;
    if ((st = w->win.reserve(sizeof(LLWin) * (size_t)B * n_t)) || (st = w->cost.reserve(sizeof(float) * B)) ||
        (st = w->order.reserve(sizeof(int32_t) * B)) || (st = w->queue.reserve(64)) ||
        (st = w->cls_off.reserve(sizeof(int32_t) * (kAllClasses + 1))))
        return st;
    if (C.nclust > 0) {
        const size_t nc = (size_t)C.nclust;
        if ((st = w->cl_x.reserve(sizeof(float) * nc * 2 * kClG * 2 * kClSlot)) ||
            (st = w->cl_part.reserve(sizeof(double) * nc * 4 * kClG)) || (st = w->cl_ninf.reserve(sizeof(double) * nc * 2 * kClG)) ||
            (st = w->cl_flag.reserve(sizeof(unsigned) * (nc * kClG * 32 + 32))))
            return st;
        bf.cl_x = w->cl_x.as<float>();
        bf.cl_part = w->cl_part.as<double>();
        bf.cl_ninf = w->cl_ninf.as<double>();
        bf.cl_flag = w->cl_flag.as<unsigned>();
    }
    bf.win = w->win.as<LLWin>();
    bf.cost = w->cost.as<float>();
    bf.order = w->order.as<int32_t>();
    bf.queue = w->queue.as<unsigned>();
    bf.cls_off = w->cls_off.as<int32_t>();
    return MJP_OK;
}

// the argument block of a call
static LLArgs ll_args(const LLContext& C, int model, int B, const mjp_obs* obs, const mjp_opts* opts,
                      const double* theta_d, const int32_t* dims_d, double* loglik_d, mjp_info* info_d,
                      const LLBufs& bf) {
    LLArgs a{};
    a.use_col = kColEnabled && col_model(model) && C.kernel[model] == MJP_LL_KERNEL_AUTO && obs->n_obs <= kColT;
    a.use_cluster = (model == MJP_MODEL_BD || model == MJP_MODEL_CASCADE2) && bf.cl_x && C.nclust > 0;
    a.theta = theta_d;
    a.dims = dims_d;
    a.T = bf.T;
    a.rec = bf.rec;
    a.win = bf.win;
    a.cost = bf.cost;
    a.order = bf.order;
    a.queue = bf.queue;
    a.cls_off = bf.cls_off;
    a.loglik = loglik_d;
    a.info = info_d;
    a.B = B;
    a.n_t = obs->n_t;
    a.n_rec = obs->n_obs;
    a.model = model;
    a.x0_1 = obs->x0[0];
    a.x0_2 = obs->x0[1];
    a.omega_factor = opts->omega_factor;
    a.tol = opts->tol;
    a.k_rule = opts->k_rule;
    a.lump = opts->lump;
    a.renorm_every = opts->truncation == MJP_CONSERVATIVE ? opts->renorm_every : 0;
    a.one_jump = opts->variant == MJP_VARIANT_PERSISTENT_ONEJUMP;
    a.k_cap = opts->k_cap;
    return a;
}

// windows, costs, classes and the order (also zeroes the class queues)
static void ll_prepare(const LLArgs& a, hipStream_t s) {
    const int nthr = a.B * a.n_t;
    hipLaunchKernelGGL(k_ll_prep, dim3((nthr + 255) / 256), dim3(256), 0, s, a);
    int P = 1;
    while (P < a.B) P <<= 1;
    const size_t sort_lds = P <= kLLMaxSort ? sizeof(unsigned long long) * P : 0;
    hipLaunchKernelGGL(k_ll_order, dim3(1), dim3(1024), sort_lds, s, a);
}

// the items of size class c of the cell kernel with shape sid: as many
// workgroups as fit on the chip (queue entry kColClasses + c)
static void ll_launch(const LLContext& C, const LLArgs& a, int cls, int sid, hipStream_t s) {
    const int grid = std::max(1, std::min(a.B, std::max(C.ncu, 1) * C.occ[a.model][sid]));
    hipLaunchKernelGGL(kLLMains[a.model][sid], dim3(grid), dim3(kLLShapes[sid].T), ll_lds(sid), s, a,
                       kColClasses + cls);
}

// the items of the cluster class (above one workgroup's LDS): zero the
// flags and the abort word, then one cooperative launch of every cluster
static mjp_status cluster_launch(const LLContext& C, const LLArgs& a, const LLBufs& bf, hipStream_t s) {
    if (!a.use_cluster) return MJP_OK;
    const int nflag = C.nclust * kClG * 32 + 32;
    hipLaunchKernelGGL(k_ll_zero_u32, dim3((nflag + 255) / 256), dim3(256), 0, s, bf.cl_flag, nflag);
    ClArgs ca{};
    ca.a = a;
    ca.xbuf = bf.cl_x;
    ca.part = bf.cl_part;
    ca.ninf = bf.cl_ninf;
    ca.wflag = bf.cl_flag;
    ca.abort_word = bf.cl_flag + (size_t)C.nclust * kClG * 32;
    ca.timeout_ticks = (uint64_t)C.wall_khz * 1000ull * 2ull;  // 2 s per wait
    ca.nclust = C.nclust;
    const void* fn = a.model == MJP_MODEL_BD ? reinterpret_cast<const void*>(k_ll_cluster<MJP_MODEL_BD>)
                                             : reinterpret_cast<const void*>(k_ll_cluster<MJP_MODEL_CASCADE2>);
    void* args[] = {&ca};
    MJP_HIP(hipLaunchCooperativeKernel(fn, dim3(C.nclust * kClG), dim3(kClT), args, cl_lds(), s));
    return MJP_OK;
}

// the items of column class cc
static void col_launch_one(const LLContext& C, const LLArgs& a, int cc, hipStream_t s) {
    const int grid = std::max(1, std::min(a.B, std::max(C.ncu, 1) * C.occ_col[cc]));
    hipLaunchKernelGGL(kColMains[cc], dim3(grid), dim3(kColT), col_lds(cc), s, a, cc);
}
// the items of every column class (nothing when the column kernel is off)
static void col_launch(const LLContext& C, const LLArgs& a, hipStream_t s) {
    if (!kColEnabled || !a.use_col) return;
    for (int cc = 0; cc < kColClasses; ++cc) col_launch_one(C, a, cc, s);
}

__global__ void k_ll_queue_reset(unsigned* q, int cls) { q[cls] = 0u; }

}  // namespace mjp

extern "C" int32_t mjp_loglik_max_states(void) { return kLLMaxStates; }

namespace mjp {

// host checks of a log-likelihood call; the records in kernel form (recs may
// be null: check only)
static mjp_status ll_check(int32_t model, int32_t B, const mjp_obs* obs, const mjp_opts* opts,
                           std::vector<LLRecord>* recs) {
    MJP_CHECK(model >= MJP_MODEL_BD && model <= MJP_MODEL_AUTOREG, MJP_E_INVALID_ARG, "unknown model %d", model);
    MJP_CHECK(B >= 0, MJP_E_INVALID_ARG, "B must be >= 0");
    mjp_status st = check_opts(opts);
    if (st) return st;
    MJP_CHECK(opts->truncation == MJP_CONSERVATIVE, MJP_E_UNSUPPORTED, "log-likelihoods use conservative truncation");
    MJP_CHECK(obs, MJP_E_INVALID_ARG, "obs is NULL");
    MJP_CHECK(obs->n_t >= 1 && obs->n_t <= kLLMaxTimes, MJP_E_INVALID_ARG, "n_t must be in [1, %d]", kLLMaxTimes);
    MJP_CHECK(obs->T_h && (obs->n_obs == 0 || obs->obs_h), MJP_E_INVALID_ARG, "null observation arrays");
    MJP_CHECK(obs->n_obs >= 0 && obs->n_obs <= kLLMaxRecords, MJP_E_INVALID_ARG, "n_obs must be in [0, %d]",
              kLLMaxRecords);
    MJP_CHECK(obs->x0[0] >= 0 && obs->x0[1] >= 0 && (model != MJP_MODEL_BD || obs->x0[1] == 0) &&
                  (model != MJP_MODEL_TWOSTATE || obs->x0[1] <= 1),
              MJP_E_INVALID_ARG, "bad initial state");
    for (int j = 0; j < obs->n_t; ++j)
        MJP_CHECK(std::isfinite(obs->T_h[j]) && obs->T_h[j] >= 0.0, MJP_E_INVALID_ARG, "T[%d] must be finite, >= 0", j);
    if (recs) recs->resize((size_t)obs->n_obs);
    for (int i = 0; i < obs->n_obs; ++i) {
        const int32_t* r = obs->obs_h + 4 * (size_t)i;
        MJP_CHECK(r[0] >= 0 && r[0] < obs->n_t, MJP_E_INVALID_ARG, "record %d: time index out of range", i);
        MJP_CHECK(r[1] >= 0 && r[2] >= 0, MJP_E_INVALID_ARG, "record %d: negative state", i);
        MJP_CHECK((model != MJP_MODEL_BD && model != MJP_MODEL_TWOSTATE) || r[2] == 0, MJP_E_INVALID_ARG,
                  "record %d: x2 must be 0 for a one-count model", i);
        MJP_CHECK(r[3] >= 1, MJP_E_INVALID_ARG, "record %d: count must be >= 1", i);
        if (recs) (*recs)[(size_t)i] = {r[0], r[1], r[2], r[3]};
    }
    return MJP_OK;
}

inline int ll_effective(const LLContext& C, int model, int cls, int n_rec) {
    const int sid = C.shape[model][cls];
    return (sid < 0 || !ll_eligible(sid, cls, n_rec)) ? kLLDefaultShape[cls] : sid;
}

// current device, checked against the table size
static mjp_status ll_device(int& dev) {
    MJP_HIP(hipGetDevice(&dev));
    MJP_CHECK(dev >= 0 && dev < kLLMaxDevices, MJP_E_UNSUPPORTED, "device %d: at most %d devices", dev, kLLMaxDevices);
    return MJP_OK;
}

// ------------------------------------------------ the allocation-free call
//
// mjp_loglik_noalloc keeps one call's tables (records, times, windows,
// costs, order, queue counters, class offsets) in this array instead of
// buffers it allocates.  The array's name is a host-side stand-in in host
// code: its device address, different on each GPU, comes from
// hipGetSymbolAddress once per device (scratch_base) and only that address
// is handed to copies and kernels.
constexpr size_t kLLScratchBytes = (size_t)6 << 20;
static __device__ __align__(256) unsigned char scratch[kLLScratchBytes];
static void* g_scratch[kLLMaxDevices];
static std::mutex g_scratch_mu;

static mjp_status scratch_base(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        MJP_CHECK(e == hipSuccess && ptr, MJP_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch[dev]);
    return MJP_OK;
}

struct LLScratchLayout {
    size_t rec, T, win, cost, order, queue, cls_off, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static LLScratchLayout scratch_layout(int B, int n_t, int n_rec) {
    LLScratchLayout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at += align256(std::max<size_t>(bytes, 1));
        return o;
    };
    L.rec = take(sizeof(LLRecord) * (size_t)n_rec);
    L.T = take(sizeof(double) * (size_t)n_t);
    L.win = take(sizeof(LLWin) * (size_t)B * n_t);
    L.cost = take(sizeof(float) * (size_t)B);
    L.order = take(sizeof(int32_t) * (size_t)B);
    L.queue = take(64);
    L.cls_off = take(sizeof(int32_t) * (kAllClasses + 1));
    L.total = at;
    return L;
}

}  // namespace mjp

extern "C" mjp_status mjp_loglik(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d,
                                 const mjp_obs* obs, const mjp_opts* opts, double* loglik_d, mjp_info* info_d,
                                 mjp_stream_t stream) {
    clear_error();
    return loglik_run(model, B, theta_d, dims_d, obs, opts, nullptr, loglik_d, info_d,
                      reinterpret_cast<hipStream_t>(stream));
}

namespace mjp {

// mjp_loglik with an optional device mask of the items to compute (the
// sampler's second stage: only proposals that passed the screen).
mjp_status loglik_run(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d, const mjp_obs* obs,
                      const mjp_opts* opts, const uint8_t* active_d, double* loglik_d, mjp_info* info_d,
                      hipStream_t s) {
    std::vector<LLRecord> recs;
    mjp_status st = ll_check(model, B, obs, opts, &recs);
    if (st) return st;
    if (B == 0) return MJP_OK;
    MJP_CHECK(theta_d && dims_d && loglik_d, MJP_E_INVALID_ARG, "null device array");
    int dev = 0;
    if ((st = ll_device(dev))) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    LLBufs bf;
    LLWork* w = nullptr;
    if ((st = ll_attrs(C, dev)) || (st = ll_obs(C, recs, obs, s, bf)) || (st = ll_work(C, s, B, obs->n_t, bf, &w)))
        return st;
    LLArgs a = ll_args(C, model, B, obs, opts, theta_d, dims_d, loglik_d, info_d, bf);
    a.active = active_d;
    ll_prepare(a, s);
    // the size classes round-robin on the caller's stream and its forked ones
    MJP_HIP(hipEventRecord(w->fork, s));
    for (int i = 0; i < kLLAux; ++i) MJP_HIP(hipStreamWaitEvent(w->aux[i], w->fork, 0));
    int rr = 0;
    auto next_stream = [&]() {
        hipStream_t t = rr == 0 ? s : w->aux[rr - 1];
        rr = (rr + 1) % (kLLAux + 1);
        return t;
    };
    // widest classes first: a class the batch leaves empty then exits at once
    // on a free chip instead of waiting, in front of a full class on its
    // stream, for CUs that an earlier class holds
    if (kColEnabled && a.use_col)
        for (int cc = kColClasses - 1; cc >= 0; --cc) col_launch_one(C, a, cc, next_stream());
    for (int c = kLLClasses - 1; c >= 0; --c) ll_launch(C, a, c, ll_effective(C, model, c, a.n_rec), next_stream());
    for (int i = 0; i < kLLAux; ++i) {
        MJP_HIP(hipEventRecord(w->join[i], w->aux[i]));
        MJP_HIP(hipStreamWaitEvent(s, w->join[i], 0));
    }
    if ((st = cluster_launch(C, a, bf, s))) return st;
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}

}  // namespace mjp

extern "C" mjp_status mjp_loglik_set_kernel(int32_t model, int32_t kernel) {
    clear_error();
    MJP_CHECK(model >= MJP_MODEL_BD && model <= MJP_MODEL_AUTOREG, MJP_E_INVALID_ARG, "unknown model %d", model);
    MJP_CHECK(kernel == MJP_LL_KERNEL_AUTO || kernel == MJP_LL_KERNEL_CELLS, MJP_E_INVALID_ARG, "unknown kernel %d",
              kernel);
    int dev = 0;
    mjp_status st = ll_device(dev);
    if (st) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    C.kernel[model] = kernel;
    return MJP_OK;
}

extern "C" mjp_status mjp_loglik_cluster_config(int32_t* clusters_h, int32_t* per_cu_h, int32_t* coop_h,
                                                int32_t* group_h, int32_t* max_states_h) {
    clear_error();
    int dev = 0;
    mjp_status st = ll_device(dev);
    if (st) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    if ((st = ll_attrs(C, dev))) return st;
    if (clusters_h) *clusters_h = C.nclust;
    if (per_cu_h) *per_cu_h = C.cl_occ;
    if (coop_h) *coop_h = C.cl_coop;
    if (group_h) *group_h = kClG;
    if (max_states_h) *max_states_h = kClMaxStates;
    return MJP_OK;
}

extern "C" int64_t mjp_loglik_noalloc_bytes(int32_t B, int32_t n_t, int32_t n_obs) {
    if (B < 0 || n_t < 0 || n_obs < 0) return -1;
    return (int64_t)scratch_layout(B, n_t, n_obs).total;
}

extern "C" int64_t mjp_loglik_noalloc_capacity(void) { return (int64_t)kLLScratchBytes; }

extern "C" mjp_status mjp_loglik_noalloc(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d,
                                         const mjp_obs* obs, const mjp_opts* opts, double* loglik_d,
                                         mjp_info* info_d, mjp_stream_t stream) {
    clear_error();
    mjp_status st = ll_check(model, B, obs, opts, nullptr);
    if (st) return st;
    if (B == 0) return MJP_OK;
    MJP_CHECK(theta_d && dims_d && loglik_d, MJP_E_INVALID_ARG, "null device array");
    const LLScratchLayout L = scratch_layout(B, obs->n_t, obs->n_obs);
    MJP_CHECK(L.total <= kLLScratchBytes, MJP_E_WORKSPACE,
              "B = %d items of %d times with %d records need %zu bytes of scratch; the allocation-free call holds %zu",
              B, obs->n_t, obs->n_obs, L.total, kLLScratchBytes);
    int dev = 0;
    if ((st = ll_device(dev))) return st;
    unsigned char* base = nullptr;
    if ((st = scratch_base(dev, &base))) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((st = ll_attrs(C, dev))) return st;
    LLBufs bf;
    bf.rec = reinterpret_cast<const LLRecord*>(base + L.rec);
    bf.T = reinterpret_cast<const double*>(base + L.T);
    bf.win = reinterpret_cast<LLWin*>(base + L.win);
    bf.cost = reinterpret_cast<float*>(base + L.cost);
    bf.order = reinterpret_cast<int32_t*>(base + L.order);
    bf.queue = reinterpret_cast<unsigned*>(base + L.queue);
    bf.cls_off = reinterpret_cast<int32_t*>(base + L.cls_off);
    // the caller's record rows have the kernels' record layout
    if (obs->n_obs)
        MJP_HIP(hipMemcpyAsync(base + L.rec, obs->obs_h, sizeof(LLRecord) * (size_t)obs->n_obs, hipMemcpyHostToDevice, s));
    MJP_HIP(hipMemcpyAsync(base + L.T, obs->T_h, sizeof(double) * (size_t)obs->n_t, hipMemcpyHostToDevice, s));
    const LLArgs a = ll_args(C, model, B, obs, opts, theta_d, dims_d, loglik_d, info_d, bf);
    ll_prepare(a, s);  // also zeroes the queue counters (no memset node)
    col_launch(C, a, s);
    for (int c = 0; c < kLLClasses; ++c) ll_launch(C, a, c, ll_effective(C, model, c, a.n_rec), s);
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}

extern "C" int32_t mjp_loglik_num_shapes(void) { return kLLNumShapes; }

extern "C" mjp_status mjp_loglik_shape(int32_t id, mjp_ll_shape* out) {
    clear_error();
    MJP_CHECK(out, MJP_E_INVALID_ARG, "out is NULL");
    MJP_CHECK(id >= 0 && id < kLLNumShapes, MJP_E_INVALID_ARG, "shape %d out of range [0, %d)", id, kLLNumShapes);
    std::memset(out, 0, sizeof(*out));
    out->threads = kLLShapes[id].T;
    out->cells = kLLShapes[id].C;
    out->max_states = ll_cap(kLLShapes[id].T, kLLShapes[id].C);
    out->lds_bytes = (int32_t)ll_lds(id);
    return MJP_OK;
}

extern "C" int32_t mjp_loglik_class_limit(int32_t cls) {
    return (cls >= 0 && cls < kLLClasses) ? kLLClassCap[cls] : 0;
}

extern "C" mjp_status mjp_loglik_set_shapes(int32_t model, const int32_t* ids) {
    clear_error();
    MJP_CHECK(model >= MJP_MODEL_BD && model <= MJP_MODEL_AUTOREG, MJP_E_INVALID_ARG, "unknown model %d", model);
    MJP_CHECK(ids, MJP_E_INVALID_ARG, "ids is NULL");
    for (int c = 0; c < kLLClasses; ++c) {
        MJP_CHECK(ids[c] >= -1 && ids[c] < kLLNumShapes, MJP_E_INVALID_ARG, "class %d: shape %d out of range", c, ids[c]);
        MJP_CHECK(ids[c] < 0 || ll_cap(kLLShapes[ids[c]].T, kLLShapes[ids[c]].C) >= kLLClassCap[c], MJP_E_INVALID_ARG,
                  "class %d: shape %d holds fewer than %d states", c, ids[c], kLLClassCap[c]);
    }
    int dev = 0;
    mjp_status st = ll_device(dev);
    if (st) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    for (int c = 0; c < kLLClasses; ++c) C.shape[model][c] = ids[c];
    return MJP_OK;
}

extern "C" mjp_status mjp_loglik_get_shapes(int32_t model, int32_t n_rec, int32_t* ids) {
    clear_error();
    MJP_CHECK(model >= MJP_MODEL_BD && model <= MJP_MODEL_AUTOREG, MJP_E_INVALID_ARG, "unknown model %d", model);
    MJP_CHECK(ids, MJP_E_INVALID_ARG, "ids is NULL");
    MJP_CHECK(n_rec >= 0 && n_rec <= kLLMaxRecords, MJP_E_INVALID_ARG, "n_rec must be in [0, %d]", kLLMaxRecords);
    int dev = 0;
    mjp_status st = ll_device(dev);
    if (st) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    for (int c = 0; c < kLLClasses; ++c) ids[c] = ll_effective(C, model, c, n_rec);
    return MJP_OK;
}

// ---- on-disk cache of the shape choices, keyed by GPU ------------------
//
// Text, one record per line:
//   mjp-loglik-shapes 1
//   gpu <architecture> <compute units> <product name, spaces as '_'>
//   table <number of shapes> <class limit 0> .. <class limit MJP_LL_CLASSES-1>
//   model <m> <shape of class 0> .. <shape of class MJP_LL_CLASSES-1>   (four lines, -1 = default)
// The gpu and table lines are the key: a file from another GPU, or from a
// build with another shape table, is refused.

static mjp_status ll_gpu_key(std::string& key) {
    int dev = 0;
    MJP_HIP(hipGetDevice(&dev));
    hipDeviceProp_t pr;
    MJP_HIP(hipGetDeviceProperties(&pr, dev));
    std::string name(pr.name), arch(pr.gcnArchName);
    for (char& ch : name)
        if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
    for (char& ch : arch)
        if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
    if (name.empty()) name = "unnamed";
    char buf[96];
    std::snprintf(buf, sizeof buf, " %d ", pr.multiProcessorCount);
    key = arch + buf + name;
    return MJP_OK;
}

static std::string ll_table_key() {
    std::string t = std::to_string(kLLNumShapes);
    for (int c = 0; c < kLLClasses; ++c) t += " " + std::to_string(kLLClassCap[c]);
    return t;
}

extern "C" mjp_status mjp_loglik_save_shapes(const char* path) {
    clear_error();
    MJP_CHECK(path && *path, MJP_E_INVALID_ARG, "path is NULL or empty");
    std::string key;
    mjp_status st = ll_gpu_key(key);
    if (st) return st;
    int dev = 0;
    if ((st = ll_device(dev))) return st;
    int shape[4][kLLClasses];
    {
        LLContext& C = ctx_for(dev);
        std::lock_guard<std::mutex> lock(C.mu);
        std::memcpy(shape, C.shape, sizeof shape);
    }
    FILE* f = std::fopen(path, "w");
    MJP_CHECK(f, MJP_E_INVALID_ARG, "cannot open %s for writing", path);
    bool ok = std::fprintf(f, "mjp-loglik-shapes 1\ngpu %s\ntable %s\n", key.c_str(), ll_table_key().c_str()) > 0;
    for (int m = 0; m < 4 && ok; ++m) {
        ok = std::fprintf(f, "model %d", m) > 0;
        for (int c = 0; c < kLLClasses && ok; ++c) ok = std::fprintf(f, " %d", shape[m][c]) > 0;
        ok = ok && std::fputc('\n', f) != EOF;
    }
    ok = (std::fclose(f) == 0) && ok;
    MJP_CHECK(ok, MJP_E_INVALID_ARG, "write to %s failed", path);
    return MJP_OK;
}

extern "C" mjp_status mjp_loglik_load_shapes(const char* path) {
    clear_error();
    MJP_CHECK(path && *path, MJP_E_INVALID_ARG, "path is NULL or empty");
    FILE* f = std::fopen(path, "r");
    MJP_CHECK(f, MJP_E_INVALID_ARG, "cannot open %s", path);
    // parse the whole file first: nothing changes unless it is complete and
    // valid (an eighth line already makes it invalid, so reading stops there)
    std::vector<std::string> lines;
    {
        char buf[512];
        while (lines.size() < 8 && std::fgets(buf, sizeof buf, f)) {
            std::string l(buf);
            while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
            lines.push_back(l);
        }
        std::fclose(f);
    }
    MJP_CHECK(lines.size() == 7 && lines[0] == "mjp-loglik-shapes 1" && lines[1].rfind("gpu ", 0) == 0 &&
                  lines[2].rfind("table ", 0) == 0,
              MJP_E_INVALID_ARG, "%s is not a shape cache", path);
    int shape[4][kLLClasses];
    for (int m = 0; m < 4; ++m) {
        int mm = -1, used = 0;
        int v[kLLClasses];
        static_assert(kLLClasses == 4, "the record below reads four classes");
        const int got = std::sscanf(lines[3 + m].c_str(), "model %d %d %d %d %d%n", &mm, &v[0], &v[1], &v[2], &v[3], &used);
        MJP_CHECK(got == 5 && mm == m && used == (int)lines[3 + m].size(), MJP_E_INVALID_ARG, "%s: bad model record %d",
                  path, m);
        for (int c = 0; c < kLLClasses; ++c) {
            MJP_CHECK(v[c] >= -1 && v[c] < kLLNumShapes &&
                          (v[c] < 0 || ll_cap(kLLShapes[v[c]].T, kLLShapes[v[c]].C) >= kLLClassCap[c]),
                      MJP_E_INVALID_ARG, "%s: model %d class %d: shape %d cannot hold the class", path, m, c, v[c]);
            shape[m][c] = v[c];
        }
    }
    MJP_CHECK(lines[2].substr(6) == ll_table_key(), MJP_E_UNSUPPORTED,
              "%s was written by a library with another shape table", path);
    std::string key;
    mjp_status st = ll_gpu_key(key);
    if (st) return st;
    MJP_CHECK(lines[1].substr(4) == key, MJP_E_UNSUPPORTED, "%s was tuned on another GPU (%s, this is %s)", path,
              lines[1].c_str() + 4, key.c_str());
    int dev = 0;
    if ((st = ll_device(dev))) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    std::memcpy(C.shape, shape, sizeof shape);
    return MJP_OK;
}

extern "C" mjp_status mjp_loglik_tune(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d,
                                      const mjp_obs* obs, const mjp_opts* opts, double* loglik_d, mjp_info* info_d,
                                      int32_t reps, mjp_ll_tune_report* report, mjp_stream_t stream) {
    clear_error();
    std::vector<LLRecord> recs;
    mjp_status st = ll_check(model, B, obs, opts, &recs);
    if (st) return st;
    MJP_CHECK(reps >= 1 && reps <= 100, MJP_E_INVALID_ARG, "reps must be in [1, 100]");
    MJP_CHECK(B >= 1, MJP_E_INVALID_ARG, "tuning needs B >= 1");
    MJP_CHECK(theta_d && dims_d && loglik_d, MJP_E_INVALID_ARG, "null device array");
    int dev = 0;
    if ((st = ll_device(dev))) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LLBufs bf;
    if ((st = ll_attrs(C, dev)) || (st = ll_obs(C, recs, obs, s, bf)) || (st = ll_work(C, s, B, obs->n_t, bf)))
        return st;
    const LLArgs a = ll_args(C, model, B, obs, opts, theta_d, dims_d, loglik_d, info_d, bf);
    ll_prepare(a, s);
    col_launch(C, a, s);  // items the column kernel or the clusters take are not tuned
    if ((st = cluster_launch(C, a, bf, s))) return st;
    int32_t off[kAllClasses + 1];
    MJP_HIP(hipMemcpyAsync(off, a.cls_off, sizeof(off), hipMemcpyDeviceToHost, s));
    MJP_HIP(hipStreamSynchronize(s));
    mjp_ll_tune_report rep;
    std::memset(&rep, 0, sizeof(rep));
    for (auto& row : rep.ms)
        for (float& v : row) v = -1.f;
    hipEvent_t e0, e1;
    MJP_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MJP_E_DEVICE, "hipEventCreate failed");
    }
    st = MJP_OK;
    for (int c = 0; c < kLLClasses && st == MJP_OK; ++c) {
        rep.items[c] = off[kColClasses + c + 1] - off[kColClasses + c];
        int best = ll_effective(C, model, c, a.n_rec);
        if (rep.items[c] > 0) {
            float best_ms = INFINITY;
            for (int sid = 0; sid < kLLNumShapes && st == MJP_OK; ++sid) {
                if (!ll_eligible(sid, c, a.n_rec)) continue;
                float t_min = INFINITY;
                for (int r = 0; r <= reps; ++r) {  // run 0 warms up
                    hipLaunchKernelGGL(k_ll_queue_reset, dim3(1), dim3(1), 0, s, a.queue, kColClasses + c);
                    if (hipEventRecord(e0, s) != hipSuccess) { st = fail(MJP_E_DEVICE, "hipEventRecord failed"); break; }
                    ll_launch(C, a, c, sid, s);
                    float ms = 0.f;
                    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        st = fail(MJP_E_DEVICE, "timing class %d shape %d failed: %s", c, sid,
                                  hipGetErrorString(hipGetLastError()));
                        break;
                    }
                    if (r > 0) t_min = std::min(t_min, ms);
                }
                rep.ms[c][sid] = t_min;
                if (t_min < best_ms) {
                    best_ms = t_min;
                    best = sid;
                }
            }
            if (st == MJP_OK) C.shape[model][c] = best;
        }
        rep.chosen[c] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    // the last run of each class was not the chosen shape's: run the chosen
    // shapes once more so the outputs are the ones mjp_loglik gives
    for (int c = 0; c < kLLClasses; ++c) {
        if (rep.items[c] == 0) continue;
        hipLaunchKernelGGL(k_ll_queue_reset, dim3(1), dim3(1), 0, s, a.queue, kColClasses + c);
        ll_launch(C, a, c, rep.chosen[c], s);
    }
    MJP_HIP(hipGetLastError());
    MJP_HIP(hipStreamSynchronize(s));
    if (report) *report = rep;
    return MJP_OK;
}

extern "C" mjp_status mjp_jump_probs(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d,
                                     const mjp_obs* obs, const int32_t* k_d, const mjp_opts* opts, double* logphi_d,
                                     double* omega_d, mjp_stream_t stream) {
    clear_error();
    std::vector<LLRecord> recs;
    mjp_status st = ll_check(model, B, obs, opts, &recs);
    if (st) return st;
    for (size_t i = 0; i < recs.size(); ++i)
        MJP_CHECK(recs[i].count == 1, MJP_E_INVALID_ARG, "record %zu: each observation has its own jump count (count 1)",
                  i);
    if (B == 0 || recs.empty()) return MJP_OK;
    MJP_CHECK(theta_d && dims_d && k_d && logphi_d, MJP_E_INVALID_ARG, "null device array");
    int dev = 0;
    if ((st = ll_device(dev))) return st;
    LLContext& C = ctx_for(dev);
    std::lock_guard<std::mutex> lock(C.mu);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    LLBufs bf;
    if ((st = ll_attrs(C, dev)) || (st = ll_obs(C, recs, obs, s, bf)) || (st = ll_work(C, s, B, obs->n_t, bf)))
        return st;
    LLArgs a = ll_args(C, model, B, obs, opts, theta_d, dims_d, nullptr, nullptr, bf);
    a.use_col = 0;  // the jump mode runs in the cell kernel
    a.n_t = 1;  // one window per item: [0, max_i k_i]
    a.kobs = k_d;
    a.phi = logphi_d;
    a.omega_out = omega_d;
    hipLaunchKernelGGL(k_jp_prep, dim3((B + 255) / 256), dim3(256), 0, s, a);
    int P = 1;
    while (P < B) P <<= 1;
    const size_t sort_lds = P <= kLLMaxSort ? sizeof(unsigned long long) * P : 0;
    hipLaunchKernelGGL(k_ll_order, dim3(1), dim3(1024), sort_lds, s, a);
    for (int c = 0; c < kLLClasses; ++c) {
        const int sid = kLLDefaultShape[c];
        const int grid = std::max(1, std::min(B, std::max(C.ncu, 1) * C.occ_jp[model][c]));
        hipLaunchKernelGGL(kJpMains[model][c], dim3(grid), dim3(kLLShapes[sid].T), ll_lds(sid), s, a, kColClasses + c);
    }
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}
