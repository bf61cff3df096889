// Krylov-subspace propagator (Method #5, Sec. 2.2.5: Algorithm ArnoldiKrylov
// and Eq. Krylov_expansion) on the GPU, in FP64.
//
// One step over [t, t + dt] from rho:
//   q_1 = rho / ||rho||;  for i = 2..kappa: q_i = q_{i-1} A orthogonalised
//   against q_1..q_{i-1} (h_{j,i-1}), h_{i,i-1} = ||q_i||, q_i /= h_{i,i-1};
//   rho(t + dt) = ||rho|| sum_i [exp(H dt)]_{i,1} q_i,
// with dt = dt_factor * kappa / max|a_nn| (the paper uses dt_factor = 2),
// shortened before each requested time so the propagation lands on it.
//
// Layout and kernels:
//  * A^T in sliced ELL (64-row slices, column-major inside a slice, FP64
//    values): the product q A is a pull over the output rows.
//  * The basis is stored unnormalised, Qraw[i] with q_i = scale[i] Qraw[i],
//    so normalising never needs a pass of its own.
//  * One Arnoldi iteration = three streaming kernels, each ending in a
//    deterministic reduction done by the last block to arrive (device-scope
//    partials and ticket, fixed summation order):
//      spmv_dot:  w = q_{i-1} A;  first projections <q_j, w>;  ||w||^2
//      orth_dot:  w -= sum_j h1_j q_j;  second projections (reorthogonalisation)
//      orth_norm: w -= sum_j h2_j q_j;  ||w||  -> h_{i,i-1}, scale[i]
//    h_{j,i-1} = h1_j + h2_j.  This is classical Gram-Schmidt with one
//    reorthogonalisation, equal to the paper's modified Gram-Schmidt in exact
//    arithmetic and as accurate in FP64; it reads each basis vector in one
//    coalesced pass instead of i dependent passes.
//  * The kappa x kappa exponential is formed by one workgroup in LDS: Taylor
//    polynomial of degree 12 (Horner) on H dt / 2^s with ||.||_1 <= 1/4,
//    then s squarings.
//  * The combination writes rho (and the output vector when the step lands
//    on a requested time) and its squared norm for the next step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gridsync.h"
#include "internal.h"

namespace mjp {

constexpr int kKB = 512;          // threads per block of the streaming kernels
constexpr int kKMax = 32;         // largest basis
constexpr int kTaylor = 12;       // Taylor degree of the small exponential
constexpr int kMaxBlocks = 256;   // grid of the streaming kernels (1 per CU)
constexpr double kBreakRel = 1e-12;

// scalar slots (FP64) of the device scalar block
constexpr int S_BETA = 0;
constexpr int S_WN2 = 1;
constexpr int S_SCALE = 8;                  // [kKMax]
constexpr int S_H1 = S_SCALE + kKMax;       // [kKMax]
constexpr int S_H2 = S_H1 + kKMax;          // [kKMax]
constexpr int S_C = S_H2 + kKMax;           // [kKMax]
constexpr int S_COUNT = S_C + kKMax;

struct KryOp {
    const int32_t* __restrict__ slice_off;
    const int32_t* __restrict__ col;
    const double* __restrict__ val;
};

// Sum of M per-thread values over the block; result for value m in red[m]
// (valid after the call for all threads).  Fixed order: wave shuffles, then
// the waves in index order.
template <int M, class P>
__device__ __forceinline__ void block_sums(double (&v)[M], P red) {
    constexpr int kWaves = kKB / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double x = v[m];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) red[m * kWaves + wave] = x;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += kKB) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += red[m * kWaves + w];
        red[m * kWaves] = s;
    }
    __syncthreads();
}

// Partials cross blocks through device-scope (agent) stores and loads,
// which the hardware performs at the device coherence point; a block's
// partial stores have completed (s_waitcnt vmcnt(0)) before its ticket
// increment, so the block that takes the last ticket reads them all.  No
// agent-scope fence is needed (one per block would write back and
// invalidate the L2 thousands of times per kernel).  The grids have at most
// kMaxBlocks blocks, so one level suffices: the last block to arrive sums
// every partial, with all of its loads issued together (a second level of
// group sums would add a ticket and a round of loads to the kernel's tail).
// (kCpolSC1 and kRsrcWord3, the device-scope cache policy of a buffer
// access and the raw-buffer descriptor word, come from gridsync.h)

__device__ __forceinline__ void put_partial(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// true in the block taking the last of `arrivals` tickets (the ticket is
// reset there)
__device__ __forceinline__ bool arrive_last(unsigned* ticket, unsigned arrivals) {
    __shared__ int is_last;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's partial stores are complete
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        is_last = (t == arrivals - 1);
        if (is_last) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return is_last;
}

// sums[m] = sum_{b < len} p[m * stride + b] for m < count: sixteen threads
// per row, each reading every sixteenth value in batches of sixteen
// device-scope loads (one batch covers 256 partials), then a fixed tree over
// the sixteen threads.
__device__ __forceinline__ void sum_rows(const double* p, size_t stride, int len, int count, double* sums) {
    const int sub = threadIdx.x & 15, slot = threadIdx.x >> 4;  // 32 rows per round
    for (int m0 = 0; m0 < count; m0 += kKB / 16) {
        const int m = m0 + slot;
        double s = 0.0;
        if (m < count) {
            const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<double*>(p + (size_t)m * stride), 0, len * 8, kRsrcWord3);
            for (int b0 = sub; b0 < len; b0 += 256) {
                double x[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)  // past len the descriptor returns 0
                    x[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                          r, (uint32_t)(b0 + 16 * u) * 8u, 0, kCpolSC1));
#pragma unroll
                for (int u = 0; u < 16; ++u) s += x[u];
            }
        }
        for (int off = 8; off > 0; off >>= 1) s += __shfl_down(s, off, 16);
        if (sub == 0 && m < count) sums[m] = s;
    }
    __syncthreads();
}

// Block partials (count values, already in red[m * waves]) -> the totals.
// Returns true in the one block that ends holding them in sums[].
struct Tree {
    double* part;  // [count][nblk]
    unsigned* tk;  // arrival ticket
};
__device__ __forceinline__ bool tree_sum(const Tree& t, const double* red, int count, double* sums) {
    const int nblk = gridDim.x, blk = blockIdx.x;
    if (threadIdx.x < count) put_partial(t.part + (size_t)threadIdx.x * nblk + blk, red[threadIdx.x * (kKB / 64)]);
    if (!arrive_last(t.tk, (unsigned)nblk)) return false;
    sum_rows(t.part, (size_t)nblk, nblk, count, sums);
    return true;
}

// ---- kernels

// Block index of the product's grid-stride loop: workgroups are dispatched
// round-robin over the 8 XCDs, so renumber them (when the grid is a multiple
// of 8) to give each XCD one band of consecutive row chunks per pass; the
// rows a product gathers (a grid line away) then mostly come from that XCD's
// own L2.
__device__ __forceinline__ int64_t kry_block() {
    const unsigned b = blockIdx.x, G = gridDim.x;
    return (G & 7u) ? (int64_t)b : (int64_t)((b & 7u) * (G >> 3) + (b >> 3));
}

// rho -> Qraw[0], ||rho||^2; last block: beta and scale[0].
__global__ __launch_bounds__(kKB) void k_kry_start(const double* __restrict__ rho, double* __restrict__ q0, int64_t n,
                                                   Tree tree, double* __restrict__ sc) {
    __shared__ double red[kKB / 64 * 1];
    double v[1] = {0.0};
    for (int64_t r = (int64_t)blockIdx.x * kKB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kKB) {
        const double x = rho[r];
        q0[r] = x;
        v[0] += x * x;
    }
    block_sums<1>(v, red);
    __shared__ double sums[1];
    if (!tree_sum(tree, red, 1, sums)) return;
    if (threadIdx.x == 0) {
        const double beta = sqrt(sums[0]);
        sc[S_BETA] = beta;
        sc[S_SCALE + 0] = beta > 0.0 ? 1.0 / beta : 0.0;
    }
}

// w = q_{i-1} A (row i of Qraw), first projections <Qraw_j, w> (j < i) and ||w||^2.
template <int I>
__global__ __launch_bounds__(kKB) void k_kry_spmv_dot(KryOp op, double* __restrict__ Q, int64_t n, Tree tree,
                                                      double* __restrict__ sc) {
    __shared__ double red[(I + 1) * (kKB / 64)];
    double v[I + 1];
#pragma unroll
    for (int m = 0; m <= I; ++m) v[m] = 0.0;
    const double* __restrict__ x = Q + (size_t)(I - 1) * n;
    const double xs = sc[S_SCALE + I - 1];
    for (int64_t r = kry_block() * kKB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kKB) {
        const int64_t s = r >> 6;
        const int lane = (int)(r & 63);
        const int32_t b = op.slice_off[s] + lane;
        const int wdt = (op.slice_off[s + 1] - op.slice_off[s]) >> 6;
        double acc = 0.0;
        int j = 0;
        for (; j + 4 <= wdt; j += 4) {  // four entries' indices and values, then their gathers
            int32_t c[4];
            double a[4], g[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = op.col[b + (j + u) * 64];
                a[u] = op.val[b + (j + u) * 64];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) g[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += a[u] * g[u];
        }
        for (; j < wdt; ++j) acc += op.val[b + j * 64] * x[op.col[b + j * 64]];
        const double w = xs * acc;
        Q[(size_t)I * n + r] = w;
#pragma unroll
        for (int jj = 0; jj < I; ++jj) v[jj] += Q[(size_t)jj * n + r] * w;
        v[I] += w * w;
    }
    block_sums<I + 1>(v, red);
    __shared__ double sums[I + 1];
    if (!tree_sum(tree, red, I + 1, sums)) return;
    if (threadIdx.x < I) sc[S_H1 + threadIdx.x] = sc[S_SCALE + threadIdx.x] * sums[threadIdx.x];
    if (threadIdx.x == 0) sc[S_WN2] = sums[I];
}

// w -= sum_j h1_j q_j; second projections.  Writes H[j][I-1] = h1_j + h2_j.
template <int I>
__global__ __launch_bounds__(kKB) void k_kry_orth_dot(double* __restrict__ Q, int64_t n, int kappa,
                                                      double* __restrict__ H, Tree tree, double* __restrict__ sc) {
    __shared__ double red[I * (kKB / 64)];
    __shared__ double coef[I];
    if (threadIdx.x < I) coef[threadIdx.x] = sc[S_H1 + threadIdx.x] * sc[S_SCALE + threadIdx.x];
    __syncthreads();
    double v[I];
#pragma unroll
    for (int m = 0; m < I; ++m) v[m] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * kKB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kKB) {
        double qj[I];
#pragma unroll
        for (int j = 0; j < I; ++j) qj[j] = Q[(size_t)j * n + r];
        double w = Q[(size_t)I * n + r];
#pragma unroll
        for (int j = 0; j < I; ++j) w -= coef[j] * qj[j];
        Q[(size_t)I * n + r] = w;
#pragma unroll
        for (int j = 0; j < I; ++j) v[j] += qj[j] * w;
    }
    block_sums<I>(v, red);
    __shared__ double sums[I];
    if (!tree_sum(tree, red, I, sums)) return;
    if (threadIdx.x < I) {
        const double h2 = sc[S_SCALE + threadIdx.x] * sums[threadIdx.x];
        sc[S_H2 + threadIdx.x] = h2;
        H[threadIdx.x * kappa + (I - 1)] = sc[S_H1 + threadIdx.x] + h2;
    }
}

// w -= sum_j h2_j q_j; ||w|| -> H[I][I-1], scale[I] (0 after a breakdown).
template <int I>
__global__ __launch_bounds__(kKB) void k_kry_orth_norm(double* __restrict__ Q, int64_t n, int kappa,
                                                       double* __restrict__ H, Tree tree, double* __restrict__ sc) {
    __shared__ double red[kKB / 64];
    __shared__ double coef[I];
    if (threadIdx.x < I) coef[threadIdx.x] = sc[S_H2 + threadIdx.x] * sc[S_SCALE + threadIdx.x];
    __syncthreads();
    double v[1] = {0.0};
    for (int64_t r = (int64_t)blockIdx.x * kKB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kKB) {
        double w = Q[(size_t)I * n + r];
#pragma unroll
        for (int j = 0; j < I; ++j) w -= coef[j] * Q[(size_t)j * n + r];
        Q[(size_t)I * n + r] = w;
        v[0] += w * w;
    }
    block_sums<1>(v, red);
    __shared__ double sums[1];
    if (!tree_sum(tree, red, 1, sums)) return;
    if (threadIdx.x == 0) {
        const double h = sqrt(sums[0]);
        const bool brk = !(h > kBreakRel * sqrt(sc[S_WN2]));
        H[I * kappa + (I - 1)] = brk ? 0.0 : h;
        sc[S_SCALE + I] = brk ? 0.0 : 1.0 / h;
    }
}

// T = exp(H dt) for the kappa x kappa Hessenberg H (any memory) by the
// workgroup, in LDS (M, T, U: kKMax^2 each): Taylor degree kTaylor by
// Horner after scaling ||H dt||_1 to <= 1/4, then the squarings.
__device__ void expm_lds(const double* H, int kappa, double dt, double* M, double* T, double* U, double* colsum,
                         int* s_sq) {
    const int kk = kappa * kappa;
    for (int e = threadIdx.x; e < kk; e += kKB) M[e] = H[e] * dt;
    __syncthreads();
    // ||M||_1 -> number of squarings so that ||M / 2^s||_1 <= 1/4
    for (int c = threadIdx.x; c < kappa; c += kKB) {
        double s = 0.0;
        for (int r = 0; r < kappa; ++r) s += fabs(M[r * kappa + c]);
        colsum[c] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double nrm = 0.0;
        for (int c = 0; c < kappa; ++c) nrm = fmax(nrm, colsum[c]);
        int s = 0;
        while (nrm > 0.25 && s < 1000) { nrm *= 0.5; ++s; }
        *s_sq = s;
    }
    __syncthreads();
    const int s = *s_sq;
    const double sc2 = ldexp(1.0, -s);
    for (int e = threadIdx.x; e < kk; e += kKB) {
        M[e] *= sc2;
        T[e] = ((e / kappa) == (e % kappa)) ? 1.0 : 0.0;  // Horner start: I
    }
    __syncthreads();
    // Horner: T = I + M T / k for k = p .. 1
    for (int k = kTaylor; k >= 1; --k) {
        const double inv = 1.0 / (double)k;
        for (int e = threadIdx.x; e < kk; e += kKB) {
            const int r = e / kappa, c = e % kappa;
            double acc = 0.0;
            for (int q = 0; q < kappa; ++q) acc += M[r * kappa + q] * T[q * kappa + c];
            U[e] = (r == c ? 1.0 : 0.0) + acc * inv;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kk; e += kKB) T[e] = U[e];
        __syncthreads();
    }
    for (int q2 = 0; q2 < s; ++q2) {
        for (int e = threadIdx.x; e < kk; e += kKB) {
            const int r = e / kappa, c = e % kappa;
            double acc = 0.0;
            for (int q = 0; q < kappa; ++q) acc += T[r * kappa + q] * T[q * kappa + c];
            U[e] = acc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kk; e += kKB) T[e] = U[e];
        __syncthreads();
    }
}

// E = exp(H dt) for the kappa x kappa Hessenberg H (one workgroup, LDS);
// c_i = beta * E[i][0] * scale[i] (the coefficient of Qraw[i]).  Clears H
// for the next step.
__global__ __launch_bounds__(kKB) void k_kry_expm(double* __restrict__ H, int kappa, double dt,
                                                  double* __restrict__ sc) {
    __shared__ double M[kKMax * kKMax], T[kKMax * kKMax], U[kKMax * kKMax];
    __shared__ double colsum[kKMax];
    __shared__ int s_sq;
    expm_lds(H, kappa, dt, M, T, U, colsum, &s_sq);
    const double beta = sc[S_BETA];
    for (int i = threadIdx.x; i < kappa; i += kKB) sc[S_C + i] = beta * T[i * kappa + 0] * sc[S_SCALE + i];
    for (int e = threadIdx.x; e < kappa * kappa; e += kKB) H[e] = 0.0;
}

// rho = sum_i c_i Qraw[i] -> Qraw[0] (next start) and out (if given);
// ||rho||^2 -> beta, scale[0] of the next step.
__global__ __launch_bounds__(kKB) void k_kry_combine(double* __restrict__ Q, int64_t n, int kappa,
                                                     double* __restrict__ out, Tree tree, double* __restrict__ sc) {
    __shared__ double red[kKB / 64];
    __shared__ double c[kKMax];
    if (threadIdx.x < kappa) c[threadIdx.x] = sc[S_C + threadIdx.x];
    __syncthreads();
    double v[1] = {0.0};
    for (int64_t r = (int64_t)blockIdx.x * kKB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kKB) {
        double x = 0.0;
        for (int i = 0; i < kappa; ++i) x += c[i] * Q[(size_t)i * n + r];
        Q[r] = x;
        if (out) out[r] = x;
        v[0] += x * x;
    }
    block_sums<1>(v, red);
    __shared__ double sums[1];
    if (!tree_sum(tree, red, 1, sums)) return;
    if (threadIdx.x == 0) {
        const double beta = sqrt(sums[0]);
        sc[S_BETA] = beta;
        sc[S_SCALE + 0] = beta > 0.0 ? 1.0 / beta : 0.0;
    }
}

__global__ void k_kry_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
    for (int64_t r = (int64_t)blockIdx.x * kKB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kKB) b[r] = a[r];
}

// ---- fused step: one cooperative launch per Krylov step
//
// The same arithmetic as the per-pass kernels above (classical Gram-Schmidt
// with one reorthogonalisation, the Taylor exponential, the combination),
// with grid barriers in place of kernel boundaries.  Block b's thread t owns
// rows r_k = b kKB + t + k G kKB (k < kKR) -- the rows and the order the
// per-pass kernels' grid-stride loops give it -- and keeps w of its rows in
// LDS (wl[k kKB + t]) through the three passes of an Arnoldi iteration,
// storing q_i once.  Every cross-block sum is: block sums (fixed order), one partial per
// block with a device-scope store, a grid barrier, then every block adds the
// G partials in the same fixed order, so all blocks hold identical totals
// and H, the scales and the exponential need no broadcast (each block keeps
// them in LDS and computes the exponential itself).  The partial buffers
// alternate between consecutive sums: a block writes sum s+1's partials only
// after the barrier of sum s, which every block passes only once done
// reading the partials of sum s-1.  Gathers of q_{i-1} (rows of other
// blocks, stored in this launch) are device-scope loads of device-scope
// stores; everything else a thread reads it wrote itself, or an earlier
// launch did.
constexpr int kKR = 8;                    // rows per thread held in registers
constexpr int kKWaves = kKB / 64;
constexpr int kKPart = kKMax + 1;         // partials per block and sum, at most
constexpr int kKBarriersPerIter = 3;

struct KryStepArgs {
    KryOp op;
    double* Q;               // kappa x n, raw basis (row 0: this step's start)
    double* out;             // this step lands on a requested time: rho here, else null
    double* part;            // [2][kKPart][G] block partials
    unsigned* bar;           // grid-barrier words, zero at the start of the solve
    unsigned* flags;         // kFlagBarrierTimeout once a barrier's deadline passed
    double* sc;              // in: S_BETA, S_SCALE + 0 of the start; out: the next step's
    int64_t n;
    double dt;
    uint64_t timeout_ticks;
    unsigned epoch0;         // grid barriers of the earlier steps of this solve
    int kappa;
};

// Device-scope 64-bit accesses through a buffer descriptor (past the range:
// loads return 0, stores are dropped).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc64(const double* p, int64_t count) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, (int)(8 * count), kRsrcWord3);
}
__device__ __forceinline__ double ld_coh(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kCpolSC1));
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_coh(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kCpolSC1);
}

// tot[m] = sum_{b < G} p[m G + b] for m < count (count <= 64, G <= 256, a
// multiple of 8): eight threads per m, thread `sub` adding partials sub,
// sub + 8, ... (all its loads issued together), then a fixed tree over the
// eight.  Every block computes the same values.
template <class P>
__device__ __forceinline__ void grid_totals(const double* p, int G, int count, P tot) {
    const int sub = threadIdx.x & 7, m = threadIdx.x >> 3;
    double s = 0.0;
    if (m < count) {
        const __amdgpu_buffer_rsrc_t r = rsrc64(p + (size_t)m * G, G);
        double x[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) x[u] = ld_coh(r, (uint32_t)(sub + 8 * u) * 8u);
#pragma unroll
        for (int u = 0; u < 32; ++u) s += x[u];
    }
    for (int off = 4; off > 0; off >>= 1) s += __shfl_down(s, off, 8);
    if (sub == 0 && m < count) tot[m] = s;
    __syncthreads();
}

// Pointers with their address space spelled out: the iteration bodies are
// separate functions, where a plain pointer would be generic and every
// access a flat instruction (which waits on both the memory and the LDS
// counters).
typedef __attribute__((address_space(3))) double* lds_d;
typedef __attribute__((address_space(1))) double* glb_d;
typedef __attribute__((address_space(1))) const int32_t* glb_ci;
typedef __attribute__((address_space(1))) const double* glb_cd;

struct KryStepCtx {
    const KryStepArgs* a;
    glb_d Q;
    glb_ci slice_off, col;
    glb_cd val;
    int64_t n;
    int G, blk, kappa;
    unsigned epoch;
    int pb;                   // partial buffer of the next sum
    bool ok;                  // false once a barrier was abandoned
    lds_d red;                // [kKPart][kKWaves]
    lds_d tot;                // [kKPart]
    lds_d Hs;                 // [kappa][kappa] (row stride kappa, as expm_lds reads it)
    lds_d scale;              // [kKMax]: 1 / ||raw q_j|| (0 after a breakdown)
    lds_d h1;                 // [kKMax]
    lds_d coef;               // [kKMax]
    lds_d wl;                 // [kKR][kKB]: this block's rows of the vector being orthogonalised
    __attribute__((address_space(3))) int32_t* rb;   // [kKR][kKB]: first entry of the row in A^T
    __attribute__((address_space(3))) int32_t* rw;   // [kKR][kKB]: entries of the row (0 past n)
};

// rows of a pass handled together (their loads in flight together): about
// 16 loads per group for the passes that read I basis vectors per row
template <int I>
constexpr int kry_group() { return I >= 16 ? 1 : (I >= 8 ? 2 : (I >= 4 ? 4 : 8)); }
constexpr int kKSpmvGroup = 4;  // rows per group of the product

__device__ __forceinline__ int64_t kry_row(const KryStepCtx& c, int k) {
    return (int64_t)c.blk * kKB + threadIdx.x + (int64_t)k * c.G * kKB;
}

// block sums of v[0..M) (fixed order) -> this block's partials -> grid
// barrier -> identical totals tot[0..M) in every block
template <int M>
__device__ __forceinline__ void kry_sum(KryStepCtx& c, double (&v)[M]) {
    block_sums<M>(v, c.red);
    double* p = c.a->part + (size_t)c.pb * kKPart * c.G;
    if (threadIdx.x < M) put_partial(p + (size_t)threadIdx.x * c.G + c.blk, c.red[threadIdx.x * kKWaves]);
    c.ok = c.ok && grid_barrier<true>(c.a->bar, ++c.epoch, logical_block(c.G), c.G, c.a->flags, c.a->timeout_ticks);
    if (c.ok) grid_totals(p, c.G, M, c.tot);
    c.pb ^= 1;
}

// Arnoldi iteration I: w = q_{I-1} A, two projections onto q_0..q_{I-1},
// norm; H column I-1, scale[I]; q_I stored (device scope).
// (one function per I, not inlined: each gets its own register allocation)
template <int I>
__device__ __noinline__ void kry_iter(KryStepCtx& c) {
    const int64_t n = c.n;
    const glb_d Q = c.Q;
    // pass 1: product (rows in groups, entry loads then gathers), then the
    // first projections (rows in groups of kry_group<I>())
    {
        const __amdgpu_buffer_rsrc_t xr = rsrc64((const double*)(Q + (size_t)(I - 1) * n), n);
        const double xs = c.scale[I - 1];
        for (int k0 = 0; k0 < kKR; k0 += kKSpmvGroup) {
            int32_t b[kKSpmvGroup], wdt[kKSpmvGroup];
            int wmax = 0;
#pragma unroll
            for (int u = 0; u < kKSpmvGroup; ++u) {
                b[u] = c.rb[(k0 + u) * kKB + threadIdx.x];
                wdt[u] = c.rw[(k0 + u) * kKB + threadIdx.x];
                wmax = max(wmax, wdt[u]);
            }
            double acc[kKSpmvGroup];
#pragma unroll
            for (int u = 0; u < kKSpmvGroup; ++u) acc[u] = 0.0;
            // four entries per row at a time; absent entries weigh 0, which
            // leaves every row's sum as the per-pass kernel forms it
            for (int j = 0; j < wmax; j += 4) {
                int32_t cc[kKSpmvGroup][4];
                double av[kKSpmvGroup][4], g[kKSpmvGroup][4];
#pragma unroll
                for (int u = 0; u < kKSpmvGroup; ++u)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const bool on = j + e < wdt[u];
                        const int at = on ? b[u] + (j + e) * 64 : 0;
                        cc[u][e] = on ? c.col[at] : 0;
                        av[u][e] = on ? c.val[at] : 0.0;
                    }
#pragma unroll
                for (int u = 0; u < kKSpmvGroup; ++u)
#pragma unroll
                    for (int e = 0; e < 4; ++e) g[u][e] = ld_coh(xr, (uint32_t)cc[u][e] * 8u);
#pragma unroll
                for (int u = 0; u < kKSpmvGroup; ++u)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[u] += av[u][e] * g[u][e];
            }
#pragma unroll
            for (int u = 0; u < kKSpmvGroup; ++u) c.wl[(k0 + u) * kKB + threadIdx.x] = xs * acc[u];
        }
        double v[I + 1];
#pragma unroll
        for (int m = 0; m <= I; ++m) v[m] = 0.0;
        constexpr int RG = kry_group<I>();
        for (int k0 = 0; k0 < kKR; k0 += RG) {
            double qj[RG][I], w[RG];
            bool live[RG];
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                const int64_t r = kry_row(c, k0 + u);
                live[u] = r < n;
                const int64_t rr = live[u] ? r : 0;
#pragma unroll
                for (int jj = 0; jj < I; ++jj) qj[u][jj] = Q[(size_t)jj * n + rr];
                w[u] = c.wl[(k0 + u) * kKB + threadIdx.x];
            }
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                if (!live[u]) continue;
#pragma unroll
                for (int jj = 0; jj < I; ++jj) v[jj] += qj[u][jj] * w[u];
                v[I] += w[u] * w[u];
            }
        }
        kry_sum<I + 1>(c, v);
        if (!c.ok) return;
        if (threadIdx.x < I) c.h1[threadIdx.x] = c.scale[threadIdx.x] * c.tot[threadIdx.x];
        if (threadIdx.x < I) c.coef[threadIdx.x] = c.h1[threadIdx.x] * c.scale[threadIdx.x];
        __syncthreads();
    }
    const double wn2 = c.tot[I];
    // pass 2: w -= sum_j h1_j q_j, second projections (the coefficients in
    // registers)
    {
        double v[I], cf[I];
#pragma unroll
        for (int m = 0; m < I; ++m) {
            v[m] = 0.0;
            cf[m] = c.coef[m];
        }
        constexpr int RG = kry_group<I>();
        for (int k0 = 0; k0 < kKR; k0 += RG) {
            double qj[RG][I], w[RG];
            bool live[RG];
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                const int64_t r = kry_row(c, k0 + u);
                live[u] = r < n;
                const int64_t rr = live[u] ? r : 0;
#pragma unroll
                for (int j = 0; j < I; ++j) qj[u][j] = Q[(size_t)j * n + rr];
                w[u] = c.wl[(k0 + u) * kKB + threadIdx.x];
            }
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                if (!live[u]) continue;
                double x = w[u];
#pragma unroll
                for (int j = 0; j < I; ++j) x -= cf[j] * qj[u][j];
                c.wl[(k0 + u) * kKB + threadIdx.x] = x;
#pragma unroll
                for (int j = 0; j < I; ++j) v[j] += qj[u][j] * x;
            }
        }
        __syncthreads();  // every thread has read coef before it is overwritten
        kry_sum<I>(c, v);
        if (!c.ok) return;
        if (threadIdx.x < I) {
            const double h2 = c.scale[threadIdx.x] * c.tot[threadIdx.x];
            c.Hs[threadIdx.x * c.kappa + (I - 1)] = c.h1[threadIdx.x] + h2;
            c.coef[threadIdx.x] = h2 * c.scale[threadIdx.x];
        }
        __syncthreads();
    }
    // pass 3: w -= sum_j h2_j q_j, norm, q_I stored
    {
        const __amdgpu_buffer_rsrc_t qr = rsrc64((const double*)(Q + (size_t)I * n), n);
        double v[1] = {0.0}, cf[I];
#pragma unroll
        for (int m = 0; m < I; ++m) cf[m] = c.coef[m];
        constexpr int RG = kry_group<I>();
        for (int k0 = 0; k0 < kKR; k0 += RG) {
            double qj[RG][I], w[RG];
            int64_t r[RG];
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                r[u] = kry_row(c, k0 + u);
                const int64_t rr = r[u] < n ? r[u] : 0;
#pragma unroll
                for (int j = 0; j < I; ++j) qj[u][j] = Q[(size_t)j * n + rr];
                w[u] = c.wl[(k0 + u) * kKB + threadIdx.x];
            }
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                if (r[u] >= n) continue;
                double x = w[u];
#pragma unroll
                for (int j = 0; j < I; ++j) x -= cf[j] * qj[u][j];
                st_coh(qr, (uint32_t)r[u] * 8u, x);
                v[0] += x * x;
            }
        }
        __syncthreads();
        kry_sum<1>(c, v);
        if (!c.ok) return;
        if (threadIdx.x == 0) {
            const double h = sqrt(c.tot[0]);
            const bool brk = !(h > kBreakRel * sqrt(wn2));
            c.Hs[I * c.kappa + (I - 1)] = brk ? 0.0 : h;
            c.scale[I] = brk ? 0.0 : 1.0 / h;
        }
        __syncthreads();
    }
}

template <int I>
__device__ __forceinline__ void kry_iter_dispatch(KryStepCtx& c, int i) {
    if constexpr (I < kKMax) {
        if (i == I) {
            kry_iter<I>(c);
            return;
        }
        kry_iter_dispatch<I + 1>(c, i);
    }
}

__global__ __launch_bounds__(kKB) void k_kry_step(KryStepArgs a) {
    __shared__ double red[kKPart * kKWaves], tot[kKPart];
    __shared__ double Hs[kKMax * kKMax], scale[kKMax], h1[kKMax], coef[kKMax];
    __shared__ double M[kKMax * kKMax], T[kKMax * kKMax], U[kKMax * kKMax], colsum[kKMax];
    __shared__ double wl[kKR * kKB];
    __shared__ int32_t rb[kKR * kKB], rw[kKR * kKB];
    __shared__ int s_sq;
    KryStepCtx c;
    c.a = &a;
    c.Q = (glb_d)a.Q;
    c.slice_off = (glb_ci)a.op.slice_off;
    c.col = (glb_ci)a.op.col;
    c.val = (glb_cd)a.op.val;
    c.n = a.n;
    c.kappa = a.kappa;
    c.G = gridDim.x;
    c.blk = blockIdx.x;
    c.epoch = a.epoch0;
    c.pb = 0;
    c.ok = true;
    c.red = (lds_d)red;
    c.tot = (lds_d)tot;
    c.Hs = (lds_d)Hs;
    c.scale = (lds_d)scale;
    c.h1 = (lds_d)h1;
    c.coef = (lds_d)coef;
    c.wl = (lds_d)wl;
    c.rb = (__attribute__((address_space(3))) int32_t*)rb;
    c.rw = (__attribute__((address_space(3))) int32_t*)rw;
    const int kappa = a.kappa;
    // each row's entries in A^T (sliced ELL: slice r / 64, lane r % 64), once per launch
    for (int k = 0; k < kKR; ++k) {
        const int64_t r = kry_row(c, k);
        int32_t b = 0, w = 0;
        if (r < a.n) {
            const int64_t sl = r >> 6;
            b = a.op.slice_off[sl] + (int32_t)(r & 63);
            w = (a.op.slice_off[sl + 1] - a.op.slice_off[sl]) >> 6;
        }
        rb[k * kKB + threadIdx.x] = b;
        rw[k * kKB + threadIdx.x] = w;
    }
    for (int e = threadIdx.x; e < kKMax * kKMax; e += kKB) Hs[e] = 0.0;
    if (threadIdx.x == 0) scale[0] = a.sc[S_SCALE + 0];
    const double beta = a.sc[S_BETA];
    __syncthreads();
    for (int i = 1; i < kappa; ++i) {
        kry_iter_dispatch<1>(c, i);
        if (!c.ok) return;
    }
    // exp(H dt) (every block, identical) and the combination of its first column
    expm_lds(Hs, kappa, a.dt, M, T, U, colsum, &s_sq);
    if (threadIdx.x < kappa) coef[threadIdx.x] = beta * T[threadIdx.x * kappa + 0] * scale[threadIdx.x];
    __syncthreads();
    const int64_t n = a.n;
    double v[1] = {0.0};
    for (int k = 0; k < kKR; ++k) {
        const int64_t r = kry_row(c, k);
        if (r < n) {
            double x = 0.0;
            for (int i = 0; i < kappa; ++i) x += coef[i] * a.Q[(size_t)i * n + r];
            a.Q[r] = x;
            if (a.out) a.out[r] = x;
            v[0] += x * x;
        }
    }
    kry_sum<1>(c, v);
    if (!c.ok) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double b2 = sqrt(tot[0]);
        a.sc[S_BETA] = b2;
        a.sc[S_SCALE + 0] = b2 > 0.0 ? 1.0 / b2 : 0.0;
    }
}

__global__ void k_kry_zero(unsigned* __restrict__ p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// per-iteration launch tables (I = 1 .. kKMax - 1)
using SpmvFn = void (*)(KryOp, double*, int64_t, Tree, double*);
using OrthFn = void (*)(double*, int64_t, int, double*, Tree, double*);

template <int... Is>
struct Tables {
    static constexpr SpmvFn spmv[sizeof...(Is)] = {k_kry_spmv_dot<Is + 1>...};
    static constexpr OrthFn dot[sizeof...(Is)] = {k_kry_orth_dot<Is + 1>...};
    static constexpr OrthFn norm[sizeof...(Is)] = {k_kry_orth_norm<Is + 1>...};
};
template <int N, int... Is>
struct MakeTables : MakeTables<N - 1, N - 1, Is...> {};
template <int... Is>
struct MakeTables<0, Is...> {
    using type = Tables<Is...>;
};
using KryTables = MakeTables<kKMax - 1>::type;

}  // namespace mjp

using namespace mjp;

struct mjp_krylov {
    int device = 0;
    int64_t n = 0;
    int32_t kappa = 20;
    double dt_factor = 2.0;
    double m_theta = 0.0;
    int32_t n_slices = 0;
    DevBuf slice_off, col, val;  // A^T sliced ELL
    DevBuf Q;                    // kappa x n FP64, unnormalised basis
    DevBuf H;                    // kappa x kappa FP64
    DevBuf part;                 // (kKMax + 1) x nblk FP64 block partials
    DevBuf sc;                   // S_COUNT FP64 scalars
    DevBuf ticket;               // arrival counter (zero between kernels)
    // fused step (one cooperative launch per step), when it fits
    bool fused = false;
    int G = 0;                   // its workgroups (a multiple of 8)
    uint64_t timeout_ticks = 0;  // deadline of one grid barrier
    DevBuf spart;                // [2][kKPart][G] block partials
    DevBuf sync;                 // kBarWords barrier words, then the flags word
};

extern "C" {

void mjp_krylov_opts_default(mjp_krylov_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->kappa = 20;
    o->dt_factor = 2.0;
}

mjp_status mjp_krylov_create(const mjp_csr* A, const mjp_krylov_opts* opts, mjp_krylov** out) {
    clear_error();
    MJP_CHECK(out, MJP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    MJP_CHECK(opts, MJP_E_INVALID_ARG, "opts is NULL");
    MJP_CHECK(opts->kappa >= 2 && opts->kappa <= kKMax, MJP_E_INVALID_ARG, "kappa must be in [2, %d]", kKMax);
    MJP_CHECK(std::isfinite(opts->dt_factor) && opts->dt_factor > 0.0, MJP_E_INVALID_ARG,
              "dt_factor must be finite and > 0");
    MJP_CHECK(opts->variant >= MJP_KRYLOV_AUTO && opts->variant <= MJP_KRYLOV_FUSED, MJP_E_INVALID_ARG,
              "variant must be MJP_KRYLOV_AUTO, _PASSES or _FUSED");
    double m_theta = 0.0;
    std::vector<double> diag;
    mjp_status st = check_generator_csr(A, 0, &m_theta, &diag);
    if (st) return st;
    const int32_t n = A->n;
    // A^T in pull form: output row m collects (source n, a_nm) for all n
    std::vector<int32_t> cnt((size_t)n, 0);
    for (int32_t r = 0; r < n; ++r)
        for (int32_t i = A->row_ptr[r]; i < A->row_ptr[r + 1]; ++i) cnt[(size_t)A->col_idx[i]]++;
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
    for (int32_t s = 0; s < n_slices; ++s) {  // padding: own row, value 0
        const int32_t w = (slice_off[(size_t)s + 1] - slice_off[(size_t)s]) / kSlice;
        for (int32_t j = 0; j < w; ++j)
            for (int32_t l = 0; l < kSlice; ++l)
                hcol[(size_t)slice_off[(size_t)s] + (size_t)j * kSlice + l] = std::min(n - 1, s * kSlice + l);
    }
    std::vector<int32_t> fill((size_t)n, 0);
    for (int32_t r = 0; r < n; ++r)
        for (int32_t i = A->row_ptr[r]; i < A->row_ptr[r + 1]; ++i) {
            const int32_t m = A->col_idx[i];
            const int32_t s = m / kSlice, l = m % kSlice;
            const size_t at = (size_t)slice_off[(size_t)s] + (size_t)fill[(size_t)m] * kSlice + l;
            hcol[at] = r;
            hval[at] = A->val[i];
            fill[(size_t)m]++;
        }

    mjp_krylov* k = new (std::nothrow) mjp_krylov();
    MJP_CHECK(k, MJP_E_DEVICE, "out of host memory");
    auto bail = [&](mjp_status s) {
        mjp_krylov_destroy(k);
        return s;
    };
    if (hipGetDevice(&k->device) != hipSuccess) return bail(fail(MJP_E_DEVICE, "no HIP device available"));
    k->n = n;
    k->kappa = opts->kappa;
    k->dt_factor = opts->dt_factor;
    k->m_theta = m_theta;
    k->n_slices = n_slices;
    const int64_t nblk = (n + kKB - 1) / kKB;
    if ((st = k->slice_off.reserve(sizeof(int32_t) * slice_off.size())) ||
        (st = k->col.reserve(sizeof(int32_t) * std::max<size_t>(total, 1))) ||
        (st = k->val.reserve(sizeof(double) * std::max<size_t>(total, 1))) ||
        (st = k->Q.reserve(sizeof(double) * (size_t)k->kappa * (size_t)n)) ||
        (st = k->H.reserve(sizeof(double) * kKMax * kKMax)) ||
        (st = k->part.reserve(sizeof(double) * (kKMax + 1) * (size_t)nblk)) ||
        (st = k->sc.reserve(sizeof(double) * S_COUNT)) ||
        (st = k->ticket.reserve(sizeof(unsigned))))
        return bail(st);
    auto up = [&](DevBuf& b, const void* h, size_t bytes) -> mjp_status {
        if (bytes) MJP_HIP(hipMemcpy(b.ptr, h, bytes, hipMemcpyHostToDevice));
        return MJP_OK;
    };
    if ((st = up(k->slice_off, slice_off.data(), sizeof(int32_t) * slice_off.size())) ||
        (st = up(k->col, hcol.data(), sizeof(int32_t) * total)) ||
        (st = up(k->val, hval.data(), sizeof(double) * total)))
        return bail(st);
    std::vector<double> zeros(kKMax * kKMax, 0.0);
    std::vector<unsigned> z32(1, 0u);
    if ((st = up(k->H, zeros.data(), sizeof(double) * kKMax * kKMax)) ||
        (st = up(k->ticket, z32.data(), sizeof(unsigned) * z32.size())))
        return bail(st);
    // the fused step (only when asked for: AUTO takes the per-pass launches,
    // which measured faster): the grid of the per-pass kernels rounded up to
    // a multiple of 8 (the barrier's groups), every workgroup co-resident, at
    // most kKR rows per thread, byte offsets of a vector within 31 bits
    if (opts->variant == MJP_KRYLOV_FUSED) {
        int coop = 0, ncu = 0, per_cu = 0, khz = 0;
        const int64_t pass_blocks = std::min<int64_t>(nblk, kMaxBlocks);
        const int64_t G = (std::max<int64_t>(pass_blocks, 8) + 7) / 8 * 8;
        bool fits = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, k->device) == hipSuccess &&
                    coop && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, k->device) == hipSuccess &&
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_kry_step),
                                                                 kKB, 0) == hipSuccess &&
                    per_cu >= 1 && G <= (int64_t)ncu * per_cu && G <= 256 && (int64_t)n <= G * kKB * kKR &&
                    8 * (int64_t)n < ((int64_t)1 << 31);
        if (!fits && opts->variant == MJP_KRYLOV_FUSED)
            return bail(fail(MJP_E_UNSUPPORTED, "the fused Krylov step does not fit this operator or device"));
        if (fits) {
            if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, k->device) != hipSuccess || khz <= 0)
                khz = 100000;
            k->fused = true;
            k->G = (int)G;
            k->timeout_ticks = (uint64_t)khz * 1000ull * 2ull;  // 2 s for one barrier
            if ((st = k->spart.reserve(sizeof(double) * 2 * kKPart * (size_t)G)) ||
                (st = k->sync.reserve(sizeof(unsigned) * (kBarWords + 1))))
                return bail(st);
        }
    }
    *out = k;
    return MJP_OK;
}

void mjp_krylov_destroy(mjp_krylov* k) {
    if (!k) return;
    int prev = 0;
    const bool restore = hipGetDevice(&prev) == hipSuccess;
    if (restore) (void)hipSetDevice(k->device);
    k->slice_off.release();
    k->col.release();
    k->val.release();
    k->Q.release();
    k->H.release();
    k->part.release();
    k->sc.release();
    k->ticket.release();
    k->spart.release();
    k->sync.release();
    if (restore) (void)hipSetDevice(prev);
    delete k;
}

int32_t mjp_krylov_n(const mjp_krylov* k) { return k ? (int32_t)k->n : 0; }

mjp_status mjp_krylov_expv(mjp_krylov* k, const double* rho0_d, int32_t n_t, const double* t_h, double* out_d,
                           mjp_krylov_info* info_h, mjp_stream_t stream) {
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
    const int kappa = k->kappa;
    // grid-stride launches: at most kMaxBlocks blocks, so each block reduces
    // once over several rows per thread
    const unsigned nblk = (unsigned)std::min<int64_t>((n + kKB - 1) / kKB, kMaxBlocks);
    double* Q = k->Q.as<double>();
    double* H = k->H.as<double>();
    const Tree tree{k->part.as<double>(), k->ticket.as<unsigned>()};
    double* sc = k->sc.as<double>();
    KryOp op{k->slice_off.as<int32_t>(), k->col.as<int32_t>(), k->val.as<double>()};

    std::vector<int> order((size_t)n_t);
    for (int j = 0; j < n_t; ++j) order[(size_t)j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return t_h[a] < t_h[b]; });
    const double dt = k->m_theta > 0.0 ? k->dt_factor * kappa / k->m_theta : INFINITY;

    hipLaunchKernelGGL(k_kry_start, dim3(nblk), dim3(kKB), 0, st, rho0_d, Q, n, tree, sc);
    KryStepArgs fa{};
    if (k->fused) {
        fa.op = op;
        fa.Q = Q;
        fa.part = k->spart.as<double>();
        fa.bar = k->sync.as<unsigned>();
        fa.flags = fa.bar + kBarWords;
        fa.sc = sc;
        fa.n = n;
        fa.timeout_ticks = k->timeout_ticks;
        fa.kappa = kappa;
        hipLaunchKernelGGL(k_kry_zero, dim3((kBarWords + 1 + 255) / 256), dim3(256), 0, st, fa.bar, kBarWords + 1);
    }
    const unsigned barriers_per_step = kKBarriersPerIter * (unsigned)(kappa - 1) + 1u;
    double tau = 0.0;
    int64_t steps = 0;
    for (int idx : order) {
        const double t = t_h[idx];
        double* outj = out_d + (size_t)idx * n;
        if (!(t - tau > 0.0) || k->m_theta == 0.0) {  // already there (t = 0, repeated time, or A = 0)
            hipLaunchKernelGGL(k_kry_copy, dim3(nblk), dim3(kKB), 0, st, Q, outj, n);
            continue;
        }
        while (t - tau > 0.0) {
            const double h = std::min(dt, t - tau);
            const bool lands = h == t - tau;
            if (k->fused) {
                fa.out = lands ? outj : nullptr;
                fa.dt = h;
                fa.epoch0 = (unsigned)steps * barriers_per_step;
                void* args[] = {&fa};
                MJP_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_kry_step), dim3(k->G), dim3(kKB),
                                                   args, 0, st));
                tau = lands ? t : tau + h;
                ++steps;
                continue;
            }
            for (int i = 1; i < kappa; ++i) {
                hipLaunchKernelGGL(KryTables::spmv[i - 1], dim3(nblk), dim3(kKB), 0, st, op, Q, n, tree, sc);
                hipLaunchKernelGGL(KryTables::dot[i - 1], dim3(nblk), dim3(kKB), 0, st, Q, n, kappa, H, tree, sc);
                hipLaunchKernelGGL(KryTables::norm[i - 1], dim3(nblk), dim3(kKB), 0, st, Q, n, kappa, H, tree, sc);
            }
            hipLaunchKernelGGL(k_kry_expm, dim3(1), dim3(kKB), 0, st, H, kappa, h, sc);
            hipLaunchKernelGGL(k_kry_combine, dim3(nblk), dim3(kKB), 0, st, Q, n, kappa, lands ? outj : nullptr, tree,
                               sc);
            tau = lands ? t : tau + h;
            ++steps;
        }
    }
    MJP_HIP(hipGetLastError());
    if (info_h) {
        std::memset(info_h, 0, sizeof(*info_h));
        info_h->m_theta = k->m_theta;
        info_h->dt = dt;
        info_h->steps = steps;
        info_h->kappa = kappa;
        info_h->fused = k->fused ? 1 : 0;
        if (k->fused && steps > 0) {
            unsigned flags = 0;
            MJP_HIP(hipMemcpyAsync(&flags, k->sync.as<unsigned>() + kBarWords, sizeof flags, hipMemcpyDeviceToHost, st));
            MJP_HIP(hipStreamSynchronize(st));
            MJP_CHECK(!(flags & kFlagBarrierTimeout), MJP_E_DEVICE, "a grid barrier of the fused Krylov step timed out");
        }
    }
    return MJP_OK;
}

}  // extern "C"
