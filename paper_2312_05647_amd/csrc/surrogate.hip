// MLP surrogate of the log-likelihood (an addition to the paper's method):
// in -> width -> ... -> width -> 1, GELU z Phi(z) between Linear layers (Phi from a rational erf form, |error| <= 1.5e-7),
// FP32 master parameters, BF16 operands on the matrix cores.
//
// Nets up to 256 wide train in three launches per step (k_mlp_fused,
// k_wgrad_all, k_adam; see the fused step below).  Wider nets, and the
// weight gradients of both, run through one MFMA GEMM kernel body
// (gemm_tile): a 64x64 output tile per workgroup, four waves of 32x32,
// FP32 accumulation.  The reduction runs in chunks of up to 256 (one
// chunk for the 256-wide layers): each thread issues all sixteen 16-byte
// loads of a chunk at once, and the chunk is staged whole in LDS in the [row][k] order the
// v_mfma_f32_16x16x32_bf16 operands want; operands stored [k][row] are
// transposed in registers in 8x8 blocks on the way.  The layers are 256
// wide, so a GEMM is a few chunks: the old 32-wide steps with a global
// round trip each were latency-bound.  The epilogue is chosen at compile
// time:
//   FWD_GELU    z = acc + b -> Z (FP32, kept for the backward pass), GELU(z) -> next input (BF16)
//   FWD_LINEAR  y = acc + b (FP32)
//   BWD_DATA    dZ_prev = acc * GELU'(Z_prev) -> BF16 (next GEMM), and the tile's
//               column sums of dZ_prev in FP32 (one partial of the previous layer's
//               bias gradient per 64 batch rows, added in a fixed order by k_adam)
//   WGRAD       split-K partial products of dW = dZ^T X (FP32), reduced in a fixed order later
// Every padded dimension is a multiple of 64 (the reduction one of 32);
// padding rows/columns carry zeros, and rows past the batch are masked in
// the loss so they contribute nothing.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "internal.h"

namespace mjp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 64, kTN = 64, kGT = 256;
constexpr int kKC = 256;          // reduction chunk staged in LDS
constexpr int kLDK = kKC + 8;     // LDS row pitch (bf16): rows 16 B apart in bank space
constexpr size_t kGemmLds = sizeof(uint16_t) * (size_t)(kTM + kTN) * kLDK;  // 67,584 B
constexpr int kMaxLayers = 9;
constexpr int kWgradChunk = 256;  // batch rows per split of the weight-gradient GEMM (one chunk)

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Standard normal CDF Phi(z) = (1 + erf(z / sqrt 2)) / 2 and density phi(z), sharing one exponential:
// erf(x) = 1 - t (a1 + a2 t + ... + a5 t^4) e^{-x^2} with t = 1 / (1 + p x) for x >= 0 (Abramowitz &
// Stegun 7.1.26, Hastings' rational form, |error| <= 1.5e-7), and e^{-x^2} at x = |z| / sqrt 2 is
// e^{-z^2/2}, the density's own factor.  Branch-free; the error is far below the BF16 rounding of the
// activations it feeds.
__device__ __forceinline__ void normal_cdf_pdf(float z, float& cdf, float& pdf) {
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
    const float e = exp2f(-0.72134752044448170f * z * z);  // e^{-z^2/2} = 2^{-z^2 log2(e) / 2}
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    const float half_erf = fmaf(-0.5f * q * t, e, 0.5f);  // erf(x) / 2
    cdf = 0.5f + copysignf(half_erf, z);
    pdf = 0.39894228040143268f * e;
}

// GELU(z) = z Phi(z) and its derivative Phi(z) + z phi(z).
__device__ __forceinline__ float gelu(float z) {
    float c, d;
    normal_cdf_pdf(z, c, d);
    return z * c;
}

__device__ __forceinline__ float gelu_grad(float z) {
    float c, d;
    normal_cdf_pdf(z, c, d);
    return fmaf(z, d, c);
}

enum { EPI_FWD_GELU = 0, EPI_FWD_LINEAR = 1, EPI_BWD_DATA = 2, EPI_WGRAD = 3 };

struct GemmArgs {
    int M, N, K;                 // padded: M, N multiples of 64, K of 32
    const uint16_t* A;           // A(m,k) = TA ? A[k*lda+m] : A[m*lda+k]
    int lda;
    const uint16_t* B;           // B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n]
    int ldb;
    int k_per_split;             // multiple of 32; gridDim.z splits
    const float* bias;           // FWD: bias[col], col < n_valid
    int n_valid;                 // columns that are real outputs
    int m_valid;                 // rows that are real batch rows (FWD_LINEAR output mask)
    float* Z;                    // FWD_GELU: out pre-activation [M x N]; BWD_DATA: in, previous layer's [M x N]
    uint16_t* H;                 // FWD_GELU: GELU out [M x N]; BWD_DATA: dZ_prev BF16 [M x N]
    float* Hf;                   // FWD_LINEAR: y [M x N]
    float* bpart;                // BWD_DATA: column sums per 64-row tile [M / 64][N]
    float* P;                    // WGRAD: partials [split][M][N]
};

// One operand tile (64 rows x a chunk of up to kKC reductions) into
// registers: eight 16-byte loads per thread, all issued together.
//   [row][k] storage: slot u covers row (tid >> 5) + 8u, k offset 8 (tid & 31)
//                     (32 lanes read one row's 512 bytes);
//   [k][row] storage: the thread owns the 8x8 block of rows rg..rg+7 and
//                     k offsets kg..kg+7 (slot u = k offset kg + u); lanes
//                     0-7 of a wave cover eight k rows, so each k row is read
//                     as one 128-byte segment by eight lanes.
// Lanes past klen (a partial last chunk) load from offset 0 of the chunk
// instead (every load is issued, none waits on a branch) and are never
// stored.
template <bool KMAJOR>
__device__ __forceinline__ void tile_load(uint4 (&v)[8], const uint16_t* __restrict__ p, int ld, int r0, int k0,
                                          int klen, int tid) {
    if (!KMAJOR) {
        const int c = (tid & 31) * 8, cc = c < klen ? c : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int r = (tid >> 5) + 8 * u;
            v[u] = *reinterpret_cast<const uint4*>(p + (size_t)(r0 + r) * ld + k0 + cc);
        }
    } else {
        const int lane = tid & 63, rg = (lane >> 3) * 8, kg = ((lane & 7) + 8 * (tid >> 6)) * 8;
        const int kc = kg < klen ? kg : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const uint4*>(p + (size_t)(k0 + kc + u) * ld + r0 + rg);
    }
}

// The registers of tile_load into LDS rows [row][k] (pitch kLDK); a [k][row]
// block is transposed first: output row c holds the eight k values of
// element c of the eight loaded vectors.
template <bool KMAJOR>
__device__ __forceinline__ void tile_store(const uint4 (&v)[8], uint16_t* __restrict__ S, int klen, int tid) {
    if (!KMAJOR) {
        const int c = (tid & 31) * 8;
        const bool on = c < klen;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (on) *reinterpret_cast<uint4*>(S + ((tid >> 5) + 8 * u) * kLDK + c) = v[u];
    } else {
        const int lane = tid & 63, rg = (lane >> 3) * 8, kg = ((lane & 7) + 8 * (tid >> 6)) * 8;
        if (kg < klen) {
            auto word = [&](int u, int w) -> uint32_t {
                return w == 0 ? v[u].x : (w == 1 ? v[u].y : (w == 2 ? v[u].z : v[u].w));
            };
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                uint32_t o[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t a = word(2 * j, c >> 1), b = word(2 * j + 1, c >> 1);
                    o[j] = (c & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
                }
                *reinterpret_cast<uint4*>(S + (rg + c) * kLDK + kg) = make_uint4(o[0], o[1], o[2], o[3]);
            }
        }
    }
}

// One 64x64 output tile (bx, by) of split bz.
template <bool TA, bool TB, int EPI>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int bx, int by, int bz, uint16_t* gemm_lds) {
    uint16_t* As = gemm_lds;               // [kTM][kLDK]
    uint16_t* Bs = gemm_lds + kTM * kLDK;  // [kTN][kLDK]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = by * kTM, n0 = bx * kTN;
    const int kbeg = bz * g.k_per_split;
    const int kend = min(g.K, kbeg + g.k_per_split);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kend; k0 += kKC) {
        const int cur = min(kKC, kend - k0);
        {
            uint4 ra[8], rb[8];
            tile_load<TA>(ra, g.A, g.lda, m0, k0, cur, tid);
            tile_load<!TB>(rb, g.B, g.ldb, n0, k0, cur, tid);
            tile_store<TA>(ra, As, cur, tid);
            tile_store<!TB>(rb, Bs, cur, tid);
        }
        __syncthreads();
        for (int ks = 0; ks < cur; ks += 32) {
            bf16x8 af[2], bfv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                af[i] = *reinterpret_cast<const bf16x8*>(As + (wm + i * 16 + (lane & 15)) * kLDK + ks + (lane >> 4) * 8);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bfv[j] = *reinterpret_cast<const bf16x8*>(Bs + (wn + j * 16 + (lane & 15)) * kLDK + ks + (lane >> 4) * 8);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    // D layout: lane holds column (lane & 15), rows 4*(lane >> 4) + r.
    // Every global operand of the epilogue is loaded before any arithmetic
    // (the bias of the lane's two columns, or the 16 pre-activations), so
    // the loads are in flight together.
    float csum[2] = {0.f, 0.f};  // BWD_DATA: this lane's rows of column j, in a fixed order
    float bj[2] = {0.f, 0.f};
    float zin[2][2][4];
    auto at_of = [&](int i, int j, int r) {
        return (size_t)(m0 + wm + i * 16 + 4 * (lane >> 4) + r) * g.N + (n0 + wn + j * 16 + (lane & 15));
    };
    if (EPI == EPI_FWD_GELU || EPI == EPI_FWD_LINEAR) {
#pragma unroll
        for (int j = 0; j < 2; ++j) bj[j] = g.bias[min(n0 + wn + j * 16 + (lane & 15), g.n_valid - 1)];
    }
    if (EPI == EPI_BWD_DATA) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) zin[i][j][r] = g.Z[at_of(i, j, r)];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                const float v = acc[i][j][r];
                const size_t at = at_of(i, j, r);
                const bool real = col < g.n_valid;
                if (EPI == EPI_FWD_GELU) {
                    const float z = real ? v + bj[j] : 0.f;
                    g.Z[at] = z;
                    g.H[at] = f2bf(real ? gelu(z) : 0.f);
                } else if (EPI == EPI_FWD_LINEAR) {
                    g.Hf[at] = real ? v + bj[j] : 0.f;
                } else if (EPI == EPI_BWD_DATA) {
                    const float d = real ? v * gelu_grad(zin[i][j][r]) : 0.f;
                    g.H[at] = f2bf(d);
                    csum[j] += d;
                } else {
                    g.P[((size_t)bz * g.M + row) * g.N + col] = v;
                }
            }
    if (EPI == EPI_BWD_DATA) {
        // column sums over the tile's 64 rows: the four row groups of a wave
        // (lanes 16 apart), then the two waves sharing the columns, via LDS
        // (free: the last chunk's barrier has passed)
        float* red = reinterpret_cast<float*>(gemm_lds);  // [2][64]
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            float t = csum[j];
            t += __shfl_xor(t, 16, 64);
            t += __shfl_xor(t, 32, 64);
            if (lane < 16) red[(wm >> 5) * 64 + wn + j * 16 + lane] = t;
        }
        __syncthreads();
        if (tid < 64) g.bpart[(size_t)by * g.N + n0 + tid] = red[tid] + red[64 + tid];
    }
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(kGT) void k_gemm(GemmArgs g) {
    extern __shared__ __attribute__((aligned(16))) uint16_t gemm_lds[];
    gemm_tile<TA, TB, EPI>(g, blockIdx.x, blockIdx.y, blockIdx.z, gemm_lds);
}

// X rows (optionally permuted) into the padded BF16 input, targets alongside.
__global__ void k_mlp_input(const float* __restrict__ x, const float* __restrict__ y, const int32_t* __restrict__ perm,
                            int base, int n_valid, int in_dim, int kpad, int Bpad, uint16_t* __restrict__ X,
                            float* __restrict__ tgt) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Bpad * kpad) return;
    const int b = idx / kpad, i = idx - b * kpad;
    float v = 0.f;
    if (b < n_valid && i < in_dim) {
        const int src = perm ? perm[base + b] : base + b;
        v = x[(size_t)src * in_dim + i];
    }
    X[idx] = f2bf(v);
    if (i == 0 && tgt) {
        float t = 0.f;
        if (b < n_valid && y) t = y[perm ? perm[base + b] : base + b];
        tgt[b] = t;
    }
}

// MSE over the n_valid real rows: dZ = 2 (y - t) / n_valid in column 0 of
// the last layer's dZ (its other columns stay zero from allocation), and
// per-block partial sums of (y - t)^2 (FP64) and of dZ's column 0 (FP32:
// the output bias gradient's partials, added in a fixed order by k_adam).
constexpr int kMseRows = 256;  // rows per block (divides every padded batch)

__global__ __launch_bounds__(kMseRows) void k_mse(const float* __restrict__ Y, int npad, const float* __restrict__ tgt,
                                                  int n_valid, int Bpad, uint16_t* __restrict__ dZ,
                                                  double* __restrict__ loss_part, float* __restrict__ bias_part) {
    __shared__ double red[kMseRows / 64];
    __shared__ float redf[kMseRows / 64];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    float d = 0.f;
    if (b < Bpad) {
        if (b < n_valid) {
            const float e = Y[(size_t)b * npad] - tgt[b];
            e2 = (double)e * (double)e;
            d = 2.f * e / (float)n_valid;
        }
        dZ[(size_t)b * npad] = f2bf(d);
    }
    for (int off = 32; off > 0; off >>= 1) {
        e2 += __shfl_down(e2, off, 64);
        d += __shfl_down(d, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = e2;
        redf[threadIdx.x >> 6] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        loss_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        bias_part[(size_t)blockIdx.x * npad] = (redf[0] + redf[1]) + (redf[2] + redf[3]);
    }
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Device copy of an epoch's permutation from mapped, coherent pinned host
// memory: an ordinary launch on the training stream, so the stream never
// hands over to the copy engine and back between epochs.
__global__ void k_copy_perm(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// MFMA B-operand fragment order of an N x K matrix (N output columns, K
// reductions; both multiples of 32): the 16 x 32 block (n/16, k/32) is 512
// consecutive values, lane (n mod 16) + 16 ((k mod 32) / 8) holding its eight
// consecutive k, so a wave loads one block as one contiguous 1 KB run.
__host__ __device__ __forceinline__ size_t frag_index(int n, int k, int K) {
    return ((size_t)(n >> 4) * (K >> 5) + (k >> 5)) * 512 + (size_t)(((n & 15) + 16 * ((k & 31) >> 3)) * 8 + (k & 7));
}

struct LayerDev {
    int in, out, kpad, npad;
    int64_t woff;      // offset of W[out][in] in the packed parameters (bias follows)
    float* P;          // weight-gradient partials [splits][npad][kpad]
    const float* bp;   // bias-gradient partials [nbp][bps] (column c = output c)
    int nbp, bps;
    uint16_t* Wbf;     // BF16 weights [npad][kpad]
    uint16_t* WbfF;    // the same in fragment order, N = npad (outputs), K = kpad (the fused forward operand)
    uint16_t* WbfB;    // ... and transposed, N = kpad, K = npad (the fused backward operand)
};

struct AdamArgs {
    int L;
    LayerDev lay[kMaxLayers];
    int splits;
    float* master;
    float* m1;
    float* m2;
    float* grad_out;   // if set: write gradients only (no update)
    float lr, beta1, beta2, eps, wd, bc1, bc2;
    int64_t total;
};

// The layer that packed parameter p belongs to (the last whose offset is <= p;
// offsets increase with the layer).  Every layer's record is read at a fixed
// index, so the loads are uniform and issue together, and the lane's record is
// picked by selects: no lane-dependent chain of loads from the argument block.
__device__ __forceinline__ LayerDev layer_of(const AdamArgs& a, int64_t p) {
    LayerDev d = a.lay[0];
#pragma unroll
    for (int j = 1; j < kMaxLayers; ++j)
        if (j < a.L && p >= a.lay[j].woff) d = a.lay[j];
    return d;
}

__global__ void k_adam(AdamArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.total) return;
    const LayerDev d = layer_of(a, p);
    // a layer holds fewer than 2^31 parameters (width <= 512, depth <= 8)
    const uint32_t q = (uint32_t)(p - d.woff);
    const uint32_t nw = (uint32_t)d.out * (uint32_t)d.in;
    float g;
    int o = -1, i = -1;
    // the partials are added in index order; eight loads are in flight at a
    // time (an out-of-range slot loads the group's first partial and adds 0)
    if (q < nw) {
        o = (int)(q / (uint32_t)d.in);
        i = (int)(q - (uint32_t)o * (uint32_t)d.in);
        g = 0.f;
        for (int s0 = 0; s0 < a.splits; s0 += 8) {
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int sl = s0 + u < a.splits ? s0 + u : s0;
                x[u] = d.P[((size_t)sl * d.npad + o) * d.kpad + i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) g += s0 + u < a.splits ? x[u] : 0.f;
        }
    } else {
        const int c = (int)(q - nw);
        g = 0.f;
        for (int k0 = 0; k0 < d.nbp; k0 += 32) {  // up to 256 partials: 32 loads in flight
            float x[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) x[u] = d.bp[(size_t)(k0 + u < d.nbp ? k0 + u : k0) * d.bps + c];
#pragma unroll
            for (int u = 0; u < 32; ++u) g += k0 + u < d.nbp ? x[u] : 0.f;
        }
    }
    if (a.grad_out) {
        a.grad_out[p] = g;
        return;
    }
    const float m = a.beta1 * a.m1[p] + (1.f - a.beta1) * g;
    const float v = a.beta2 * a.m2[p] + (1.f - a.beta2) * g * g;
    a.m1[p] = m;
    a.m2[p] = v;
    const float mh = m / a.bc1, vh = v / a.bc2;
    float w = a.master[p];
    w -= a.lr * (mh / (sqrtf(vh) + a.eps) + a.wd * w);
    a.master[p] = w;
    if (o >= 0) {
        const uint16_t h = f2bf(w);
        d.Wbf[(size_t)o * d.kpad + i] = h;
        d.WbfF[frag_index(o, i, d.kpad)] = h;
        d.WbfB[frag_index(i, o, d.npad)] = h;
    }
}

// BF16 padded copies of all weights from the masters (after create/set/load).
__global__ void k_refresh_bf16(AdamArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.total) return;
    const LayerDev d = layer_of(a, p);
    const int64_t q = p - d.woff;
    if (q < (int64_t)d.out * d.in) {
        const int o = (int)(q / d.in), i = (int)(q - (int64_t)o * d.in);
        const uint16_t h = f2bf(a.master[p]);
        d.Wbf[(size_t)o * d.kpad + i] = h;
        d.WbfF[frag_index(o, i, d.kpad)] = h;
        d.WbfB[frag_index(i, o, d.npad)] = h;
    }
}

__global__ void k_copy_col0(const float* __restrict__ Y, int npad, int n, float* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) out[b] = Y[(size_t)b * npad];
}

// ---- fused training step: one workgroup per 16 batch rows -------------
//
// For nets no wider than 256 a workgroup carries its rows through the whole
// network: input gather, every hidden layer forward (pre-activations kept in
// LDS for the backward pass), the output layer and the squared-error loss,
// then the backward-data products down to the first layer's output
// gradient.  Activations never leave LDS between layers; each layer's input
// (forward) and output gradient (backward) is also written to global memory
// in BF16 for the weight-gradient launch.  Wave w owns output column tiles w
// and w + 8 (16 columns each) of every product and streams its slice of the
// weights straight into registers as MFMA B operands -- no LDS staging, the
// slice is private to the wave.  The forward products read W, the backward
// ones W^T, both kept by the optimiser in B-operand fragment order
// (frag_index), so each load of a wave is one contiguous 1 KB run.
//
// The next product's slice is loaded while the current one computes.  The
// wave's memory counter covers loads and stores alike, and with both in
// flight a wait for one load is a wait for everything, so each pass first
// takes its own (already loaded) slice, then issues the next slice's loads,
// then the MFMAs, and only then the global stores of the previous pass's
// output: the stores are the youngest operations when the pass ends, and the
// prefetch stays in flight across the MFMAs.
constexpr int kFThreads = 512;    // eight waves
constexpr int kFMaxW = 256;       // widest hidden layer: two column tiles per wave
constexpr int kFMaxKS = kFMaxW / 32;
constexpr int kFMinRows = 16;     // ... and at least (sizes the per-workgroup partials)

struct FusedArgs {
    int L, width, in_dim, kpad0;
    int n_valid, base;                // rows base .. base + n_valid - 1 of x (and y) are real
    const float* x;                   // [n][in_dim]
    const float* y;                   // targets [n] (training)
    const int32_t* perm;              // optional row permutation
    const float* master;              // FP32 parameters (the biases are read from here)
    int64_t boff[kMaxLayers];         // offset of layer l's bias in master
    const uint16_t* W[kMaxLayers];    // BF16 [npad_l][kpad_l]
    const uint16_t* WF[kMaxLayers];   // the same, B-operand fragment order (N = npad_l, K = kpad_l)
    const uint16_t* WB[kMaxLayers];   // transposed, fragment order (N = kpad_l, K = npad_l)
    uint16_t* X[kMaxLayers];          // layer inputs [Bpad][kpad_l] (training)
    uint16_t* dZ[kMaxLayers];         // output gradients [Bpad][npad_l] (training)
    float* bpart[kMaxLayers];         // bias-gradient partials [Bpad / MT][npad_l] (training)
    double* lossp;                    // squared-error partials [Bpad / MT] (training)
    float* yout;                      // inference: outputs of the n_valid rows
};

// LDS of the fused step at MT rows per workgroup: pre-activations of the
// L - 1 hidden layers (FP32, training only), two BF16 row buffers
// [MT][width + 8], the output layer's weights (FP32), and MT rows of loss
// scratch.
__host__ __device__ constexpr size_t fused_lds_bytes(bool train, int L, int width, int MT) {
    return (train ? sizeof(float) * (size_t)(L - 1) * MT * width : 0) +
           sizeof(uint16_t) * 2 * (size_t)MT * (width + 8) + sizeof(float) * (size_t)width +
           (sizeof(double) + 3 * sizeof(float)) * (size_t)MT;
}

// keeps a register's load complete here (an empty use the compiler must wait for)
__device__ __forceinline__ void take(const uint4& v) {
    asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

template <bool TRAIN, int MR>
__global__ __launch_bounds__(kFThreads) void k_mlp_fused(FusedArgs a) {
    constexpr int MT = 16 * MR;       // batch rows of the workgroup
    extern __shared__ __attribute__((aligned(16))) char flds[];
    const int L = a.L, W = a.width, P = W + 8, NT = W / 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row0 = blockIdx.x * MT;
    float* Zs = reinterpret_cast<float*>(flds);                                     // [L-1][MT][W]
    uint16_t* Hb = reinterpret_cast<uint16_t*>(Zs + (TRAIN ? (L - 1) * MT * W : 0));  // [2][MT][P]
    float* wl = reinterpret_cast<float*>(Hb + 2 * MT * P);                          // output weights [W]
    double* se = reinterpret_cast<double*>(wl + W);                                 // squared errors [MT]
    float* tg = reinterpret_cast<float*>(se + MT);                                  // targets [MT]
    float* dyb = tg + MT;                                                           // BF16-rounded dy [MT]
    float* dyf = dyb + MT;                                                          // dy [MT]

    // input rows (BF16, zero padded to kpad0) into buffer 0 and, training, X[0]
    for (int e = tid; e < MT * a.kpad0; e += kFThreads) {
        const int r = e / a.kpad0, i = e - r * a.kpad0, b = row0 + r;
        float v = 0.f;
        if (b < a.n_valid && i < a.in_dim) {
            const int src = a.perm ? a.perm[a.base + b] : a.base + b;
            v = a.x[(size_t)src * a.in_dim + i];
        }
        const uint16_t h = f2bf(v);
        Hb[r * P + i] = h;
        if (TRAIN) a.X[0][(size_t)b * a.kpad0 + i] = h;
    }
    if (TRAIN && tid < MT) {
        const int b = row0 + tid;
        tg[tid] = b < a.n_valid ? a.y[a.perm ? a.perm[a.base + b] : a.base + b] : 0.f;
    }
    for (int c = tid; c < W; c += kFThreads) wl[c] = bf2f(a.W[L - 1][c]);
    const float blast = a.master[a.boff[L - 1]];

    // product p: forward layer p for p < L - 1, then backward through layer
    // 2L - 3 - p (its W^T) for the training passes
    auto geom = [&](int p, int& l, int& K, bool& fwd) {
        fwd = p < L - 1;
        l = fwd ? p : 2 * L - 3 - p;
        K = (fwd && p == 0) ? a.kpad0 : W;
    };
    // Every load is issued unconditionally (a load under a branch leaves the
    // compiler unsure which are still in flight, and it then waits for all):
    // a tile past the layer's width reads its last tile again, a reduction
    // step past K reads step 0 again, and neither is used.
    auto wload = [&](int p, uint4 (&wr)[2][kFMaxKS], float (&br)[2]) {
        int l, K;
        bool fwd;
        geom(p, l, K, fwd);
        const uint16_t* M = fwd ? a.WF[l] : a.WB[l];
        const int KS = K >> 5;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int tile = min(wave + 8 * t, NT - 1);
            const uint16_t* q = M + (size_t)tile * KS * 512 + lane * 8;
#pragma unroll
            for (int ks = 0; ks < kFMaxKS; ++ks)
                wr[t][ks] = *reinterpret_cast<const uint4*>(q + (ks < KS ? ks : 0) * 512);
            br[t] = a.master[a.boff[l] + tile * 16 + (lane & 15)];  // used by the forward products only
        }
    };
    auto wtake = [&](const uint4 (&wr)[2][kFMaxKS], const float (&br)[2]) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
            for (int ks = 0; ks < kFMaxKS; ++ks) take(wr[t][ks]);
            asm volatile("" ::"v"(br[t]));
        }
        asm volatile("" ::: "memory");  // the next slice's loads stay behind this wait
    };
    // MT rows of a buffer to global rows row0.. of dst (16-byte stores)
    auto spill = [&](const uint16_t* from, uint16_t* dst) {
        const int per = W / 8;
        for (int e = tid; e < MT * per; e += kFThreads) {
            const int r = e / per, c8 = (e - r * per) * 8;
            *reinterpret_cast<uint4*>(dst + (size_t)(row0 + r) * W + c8) =
                *reinterpret_cast<const uint4*>(from + r * P + c8);
        }
    };
    uint16_t* pend = nullptr;  // global destination of the rows in the current input buffer
    auto mpass = [&](int p, const uint4 (&wr)[2][kFMaxKS], const float (&br)[2]) {
        int l, K;
        bool fwd;
        geom(p, l, K, fwd);
        const uint16_t* Ain = Hb + (p & 1) * MT * P;
        uint16_t* Hout = Hb + ((p + 1) & 1) * MT * P;
        floatx4 acc[MR][2];
#pragma unroll
        for (int i = 0; i < MR; ++i)
#pragma unroll
            for (int t = 0; t < 2; ++t) acc[i][t] = floatx4{0.f, 0.f, 0.f, 0.f};
        // reduction steps past K (the first layer's) multiply zeros
#pragma unroll
        for (int ks = 0; ks < kFMaxKS; ++ks) {
            const bool on = ks * 32 < K;
            bf16x8 av[MR];
#pragma unroll
            for (int i = 0; i < MR; ++i) {
                const uint4 v = *reinterpret_cast<const uint4*>(Ain + (i * 16 + (lane & 15)) * P + ks * 32 + 8 * (lane >> 4));
                av[i] = __builtin_bit_cast(bf16x8, on ? v : make_uint4(0u, 0u, 0u, 0u));
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < MR; ++i)
                    acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        av[i], __builtin_bit_cast(bf16x8, on ? wr[t][ks] : make_uint4(0u, 0u, 0u, 0u)), acc[i][t], 0,
                        0, 0);
        }
        asm volatile("" ::: "memory");
        if (TRAIN && pend) spill(Ain, pend);  // the previous pass's output, behind the MFMAs
        // D layout: lane holds column (lane & 15) of a tile, rows 4 (lane >> 4) + r
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int tile = wave + 8 * t;
            if (tile >= NT) continue;
            const int c = tile * 16 + (lane & 15);
            if (fwd) {
#pragma unroll
                for (int i = 0; i < MR; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = i * 16 + 4 * (lane >> 4) + r;
                        const float z = acc[i][t][r] + br[t];
                        if (TRAIN) Zs[(l * MT + row) * W + c] = z;
                        Hout[row * P + c] = f2bf(gelu(z));
                    }
            } else {
                float cs = 0.f;
#pragma unroll
                for (int i = 0; i < MR; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = i * 16 + 4 * (lane >> 4) + r;
                        const float d = acc[i][t][r] * gelu_grad(Zs[((l - 1) * MT + row) * W + c]);
                        Hout[row * P + c] = f2bf(d);
                        cs += d;
                    }
                cs += __shfl_xor(cs, 16, 64);
                cs += __shfl_xor(cs, 32, 64);
                if (lane < 16) a.bpart[l - 1][(size_t)blockIdx.x * W + c] = cs;
            }
        }
        __syncthreads();
        pend = TRAIN ? (fwd ? a.X[l + 1] : a.dZ[l - 1]) : nullptr;
    };
    // output layer (one column, VALU), loss and, training, the gradient
    // through it into layer L - 2's output gradient
    auto output_layer = [&]() {
        constexpr int LPR = kFThreads / MT;  // lanes per row
        uint16_t* Hin = Hb + ((L - 1) & 1) * MT * P;
        const int r = tid / LPR, j = tid % LPR;
        float sacc = 0.f;
#pragma unroll
        for (int u = 0; u < kFMaxW / LPR; ++u) {  // independent loads, one accumulation order
            const int k = j + u * LPR;
            const float hv = k < W ? bf2f(Hin[r * P + k]) : 0.f;
            sacc = fmaf(hv, k < W ? wl[k] : 0.f, sacc);
        }
#pragma unroll
        for (int m = LPR / 2; m > 0; m >>= 1) sacc += __shfl_xor(sacc, m, LPR);
        const float yv = sacc + blast;
        const bool real = row0 + r < a.n_valid;
        if (!TRAIN) {
            if (j == 0 && real) a.yout[row0 + r] = yv;
            return;
        }
        if (j == 0) {
            const float e = yv - tg[r];
            const float d = real ? 2.f * e / (float)a.n_valid : 0.f;
            const uint16_t db = f2bf(d);
            se[r] = real ? (double)e * (double)e : 0.0;
            dyf[r] = d;
            dyb[r] = bf2f(db);
            a.dZ[L - 1][(size_t)(row0 + r) * 64] = db;
        }
        spill(Hin, pend);  // this layer's input, before the buffer is reused
        __syncthreads();   // every row's y is formed and stored: Hin can be overwritten
        if (wave == 0) {  // the rows' squared errors and dy, a fixed shuffle tree
            double s2 = lane < MT ? se[lane] : 0.0;
            float sd = lane < MT ? dyf[lane] : 0.f;
#pragma unroll
            for (int m = MT / 2; m > 0; m >>= 1) {
                s2 += __shfl_xor(s2, m, 64);
                sd += __shfl_xor(sd, m, 64);
            }
            if (lane == 0) {
                a.lossp[blockIdx.x] = s2;
                a.bpart[L - 1][(size_t)blockIdx.x * 64] = sd;
            }
        }
        float* Zl = Zs + (size_t)(L - 2) * MT * W;  // becomes layer L - 2's output gradient (FP32)
        for (int e = tid; e < MT * W; e += kFThreads) {
            const int rr = e / W, c = e - rr * W;
            const float d = (dyb[rr] * wl[c]) * gelu_grad(Zl[e]);
            Zl[e] = d;
            Hin[rr * P + c] = f2bf(d);
        }
        __syncthreads();
        for (int c = tid; c < W; c += kFThreads) {
            float cs = 0.f;
            for (int q = 0; q < MT; ++q) cs += Zl[q * W + c];
            a.bpart[L - 2][(size_t)blockIdx.x * W + c] = cs;
        }
        pend = a.dZ[L - 2];
    };

    const int NP = TRAIN ? 2 * L - 3 : L - 1;
    uint4 wA[2][kFMaxKS], wB[2][kFMaxKS];
    float bA[2] = {0.f, 0.f}, bB[2] = {0.f, 0.f};
    wload(0, wA, bA);
    __syncthreads();  // input rows and output weights staged
    auto stage = [&](int p, const uint4 (&cur)[2][kFMaxKS], const float (&bc)[2], uint4 (&nxt)[2][kFMaxKS],
                     float (&bn)[2]) {
        wtake(cur, bc);
        if (p + 1 < NP) wload(p + 1, nxt, bn);
        mpass(p, cur, bc);
        if (p == L - 2) output_layer();
    };
    for (int p = 0; p < NP; p += 2) {
        stage(p, wA, bA, wB, bB);
        if (p + 1 >= NP) break;
        stage(p + 1, wB, bB, wA, bA);
    }
    if (TRAIN) spill(Hb + (NP & 1) * MT * P, pend);  // the first layer's output gradient
}

// Weight gradients of every layer in one launch: the split-K tiles of all
// layers' dW = dZ^T X, laid end to end in the grid, then one block per 64
// bias columns of each layer adding that layer's per-workgroup bias partials
// (four interleaved strided sums, 16 loads in flight each, joined in a fixed
// order) into one bias gradient.
struct WgradAll {
    int L;
    int start[kMaxLayers + 1];   // first block of layer l's weight tiles; start[L]: the bias blocks
    int bstart[kMaxLayers + 1];  // first bias block of layer l, counted from start[L]
    GemmArgs g[kMaxLayers];
    const float* bpart[kMaxLayers];  // [nbp][npad_l]
    float* bgrad[kMaxLayers];        // [npad_l]
    int nbp;
};

__global__ __launch_bounds__(kGT) void k_wgrad_all(WgradAll w) {
    extern __shared__ __attribute__((aligned(16))) uint16_t gemm_lds[];
    int b = blockIdx.x;
    if (b >= w.start[w.L]) {
        b -= w.start[w.L];
        int l = 0;
        while (l + 1 < w.L && b >= w.bstart[l + 1]) ++l;
        const int npad = w.g[l].M;  // the layer's padded outputs
        const int c = (b - w.bstart[l]) * 64 + (threadIdx.x & 63), grp = threadIdx.x >> 6;
        const float* bp = w.bpart[l];
        float acc = 0.f;
        for (int k0 = grp; k0 < w.nbp; k0 += 4 * 16) {
            float x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int k = k0 + 4 * u;
                x[u] = bp[(size_t)(k < w.nbp ? k : grp) * npad + c];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += k0 + 4 * u < w.nbp ? x[u] : 0.f;
        }
        float* red = reinterpret_cast<float*>(gemm_lds);
        red[threadIdx.x] = acc;
        __syncthreads();
        if (threadIdx.x < 64) w.bgrad[l][c] = (red[threadIdx.x] + red[64 + threadIdx.x]) + (red[128 + threadIdx.x] + red[192 + threadIdx.x]);
        return;
    }
    int l = 0;
    while (l + 1 < w.L && b >= w.start[l + 1]) ++l;
    b -= w.start[l];
    const GemmArgs& g = w.g[l];
    const int nx = g.N / kTN, ny = g.M / kTM;
    gemm_tile<true, false, EPI_WGRAD>(g, b % nx, (b / nx) % ny, b / (nx * ny), gemm_lds);
}

}  // namespace mjp

using namespace mjp;

struct mjp_surrogate {
    mjp_mlp_cfg cfg{};
    int device = 0;
    int L = 0;
    int in[kMaxLayers], out[kMaxLayers], kpad[kMaxLayers], npad[kMaxLayers];
    int64_t woff[kMaxLayers + 1];
    int64_t total = 0;
    int Bmax = 0, splits = 0;
    int64_t step = 0;
    DevBuf master, m1, m2, gradbuf;
    DevBuf wbf[kMaxLayers], wbfF[kMaxLayers], wbfB[kMaxLayers], P[kMaxLayers];
    bool fused = false;        // nets up to 256 wide: the three-launch training step
    int mt = 16;               // its batch rows per workgroup
    DevBuf X[kMaxLayers + 1];  // BF16 inputs of each layer [Bmax x kpad]; X[L] unused
    DevBuf Z[kMaxLayers];      // FP32 pre-activations [Bmax x npad]
    DevBuf dZ[kMaxLayers];     // BF16 output gradients [Bmax x npad]
    DevBuf bpart[kMaxLayers];  // bias-gradient partials [Bmax / 16][npad] (one per 16 rows at most)
    DevBuf bgrad[kMaxLayers];  // fused step: the bias gradients [npad], from the partials
    DevBuf Y, tgt, lossp, perm;
};

namespace mjp {

static int round_up(int v, int m) { return (v + m - 1) / m * m; }

static mjp_status surrogate_alloc(mjp_surrogate* s, int Bmax, hipStream_t st_) {
    if (Bmax <= s->Bmax) return MJP_OK;
    s->Bmax = Bmax;
    s->splits = std::max(1, Bmax / kWgradChunk);
    mjp_status st;
    for (int l = 0; l < s->L; ++l) {
        if ((st = s->X[l].reserve(sizeof(uint16_t) * (size_t)Bmax * s->kpad[l])) ||
            (st = s->Z[l].reserve(sizeof(float) * (size_t)Bmax * s->npad[l])) ||
            (st = s->dZ[l].reserve(sizeof(uint16_t) * (size_t)Bmax * s->npad[l])) ||
            (st = s->bpart[l].reserve(sizeof(float) * (size_t)(Bmax / kFMinRows) * s->npad[l])) ||
            (st = s->bgrad[l].reserve(sizeof(float) * (size_t)s->npad[l])) ||
            (st = s->P[l].reserve(sizeof(float) * (size_t)s->splits * s->npad[l] * s->kpad[l])))
            return st;
    }
    if ((st = s->Y.reserve(sizeof(float) * (size_t)Bmax * s->npad[s->L - 1])) ||
        (st = s->tgt.reserve(sizeof(float) * (size_t)Bmax)) ||
        (st = s->lossp.reserve(sizeof(double) * (size_t)(Bmax / kFMinRows))))
        return st;
    // the loss kernel writes only column 0 of the last layer's dZ: the
    // padding columns are cleared once per allocation
    const size_t words = (size_t)Bmax * s->npad[s->L - 1] / 2;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st_,
                       s->dZ[s->L - 1].as<uint32_t>(), words);
    if (hipGetLastError() != hipSuccess) return fail(MJP_E_DEVICE, "clearing the output gradient failed");
    return MJP_OK;
}

static AdamArgs adam_args(mjp_surrogate* s) {
    AdamArgs a{};
    a.L = s->L;
    for (int l = 0; l < s->L; ++l) {
        a.lay[l].in = s->in[l];
        a.lay[l].out = s->out[l];
        a.lay[l].kpad = s->kpad[l];
        a.lay[l].npad = s->npad[l];
        a.lay[l].woff = s->woff[l];
        a.lay[l].P = s->P[l].as<float>();
        a.lay[l].bp = s->bpart[l].as<float>();
        a.lay[l].nbp = 0;
        a.lay[l].bps = s->npad[l];
        a.lay[l].Wbf = s->wbf[l].as<uint16_t>();
        a.lay[l].WbfF = s->wbfF[l].as<uint16_t>();
        a.lay[l].WbfB = s->wbfB[l].as<uint16_t>();
    }
    a.splits = s->splits;
    a.master = s->master.as<float>();
    a.m1 = s->m1.as<float>();
    a.m2 = s->m2.as<float>();
    a.total = s->total;
    return a;
}

// The GEMM's LDS chunk is above the default 64 KB limit: raise it once per
// instantiation (the same four the dispatcher below launches).
static hipError_t gemm_lds_limits() {
    const void* fns[] = {reinterpret_cast<const void*>(k_gemm<false, true, EPI_FWD_GELU>),
                         reinterpret_cast<const void*>(k_gemm<false, true, EPI_FWD_LINEAR>),
                         reinterpret_cast<const void*>(k_gemm<false, false, EPI_BWD_DATA>),
                         reinterpret_cast<const void*>(k_gemm<true, false, EPI_WGRAD>)};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static void launch_gemm(bool TA, bool TB, int epi, const GemmArgs& g, int splits, hipStream_t st) {
    static const hipError_t lds_ok = gemm_lds_limits();  // a failure surfaces as a launch error
    (void)lds_ok;
    const dim3 grid(g.N / kTN, g.M / kTM, splits);
#define MJP_G(ta, tb, e) \
    if (TA == ta && TB == tb && epi == e) { hipLaunchKernelGGL((k_gemm<ta, tb, e>), grid, dim3(kGT), kGemmLds, st, g); return; }
    MJP_G(false, true, EPI_FWD_GELU)
    MJP_G(false, true, EPI_FWD_LINEAR)
    MJP_G(false, false, EPI_BWD_DATA)
    MJP_G(true, false, EPI_WGRAD)
#undef MJP_G
}

// forward pass of rows already in X[0]: Y = MLP(X[0]) (n_valid rows real)
static void forward(mjp_surrogate* s, int Bpad, int n_valid, hipStream_t st) {
    for (int l = 0; l < s->L; ++l) {
        GemmArgs g{};
        g.M = Bpad;
        g.N = s->npad[l];
        g.K = s->kpad[l];
        g.A = s->X[l].as<uint16_t>();
        g.lda = s->kpad[l];
        g.B = s->wbf[l].as<uint16_t>();
        g.ldb = s->kpad[l];
        g.k_per_split = g.K;
        g.bias = s->master.as<float>() + s->woff[l] + (int64_t)s->out[l] * s->in[l];
        g.n_valid = s->out[l];
        g.m_valid = n_valid;
        if (l + 1 < s->L) {
            g.Z = s->Z[l].as<float>();
            g.H = s->X[l + 1].as<uint16_t>();
            launch_gemm(false, true, EPI_FWD_GELU, g, 1, st);
        } else {
            g.Hf = s->Y.as<float>();
            launch_gemm(false, true, EPI_FWD_LINEAR, g, 1, st);
        }
    }
}

// backward pass after forward + loss (dZ[L-1] set): fills P and gb
static void backward(mjp_surrogate* s, int Bpad, hipStream_t st) {
    for (int l = s->L - 1; l >= 0; --l) {
        GemmArgs w{};
        w.M = s->npad[l];
        w.N = s->kpad[l];
        w.K = Bpad;
        w.A = s->dZ[l].as<uint16_t>();
        w.lda = s->npad[l];
        w.B = s->X[l].as<uint16_t>();
        w.ldb = s->kpad[l];
        const int splits = std::max(1, Bpad / kWgradChunk);
        w.k_per_split = Bpad / splits;
        w.P = s->P[l].as<float>();
        launch_gemm(true, false, EPI_WGRAD, w, splits, st);  // the reduction reads only these splits
        if (l > 0) {
            GemmArgs d{};
            d.M = Bpad;
            d.N = s->kpad[l];
            d.K = s->npad[l];
            d.A = s->dZ[l].as<uint16_t>();
            d.lda = s->npad[l];
            d.B = s->wbf[l].as<uint16_t>();
            d.ldb = s->kpad[l];
            d.k_per_split = d.K;
            d.n_valid = s->in[l];
            d.Z = s->Z[l - 1].as<float>();
            d.H = s->dZ[l - 1].as<uint16_t>();
            d.bpart = s->bpart[l - 1].as<float>();
            launch_gemm(false, false, EPI_BWD_DATA, d, 1, st);
        }
    }
}

static void load_rows(mjp_surrogate* s, const float* x, const float* y, const int32_t* perm, int base, int n_valid,
                      int Bpad, hipStream_t st) {
    const int tot = Bpad * s->kpad[0];
    hipLaunchKernelGGL(k_mlp_input, dim3((tot + 255) / 256), dim3(256), 0, st, x, y, perm, base, n_valid, s->in[0],
                       s->kpad[0], Bpad, s->X[0].as<uint16_t>(), s->tgt.as<float>());
}

// loss partials go to loss_part[Bpad / kMseRows]
static void loss_grad(mjp_surrogate* s, int n_valid, int Bpad, double* loss_part, hipStream_t st) {
    hipLaunchKernelGGL(k_mse, dim3(Bpad / kMseRows), dim3(kMseRows), 0, st, s->Y.as<float>(), s->npad[s->L - 1],
                       s->tgt.as<float>(), n_valid, Bpad, s->dZ[s->L - 1].as<uint16_t>(), loss_part,
                       s->bpart[s->L - 1].as<float>());
}

// Split-K count of the weight-gradient products at padded batch Bpad: one
// split per 256 rows on the per-layer path; at most kFusedSplits on the fused
// one (fewer partials for the optimiser to add, each split a longer reduction).
constexpr int kFusedSplits = 8;
static int wgrad_splits(const mjp_surrogate* s, int Bpad) {
    const int sp = std::max(1, Bpad / kWgradChunk);
    return s->fused ? std::min(sp, kFusedSplits) : sp;
}

// Adam arguments of one training step at padded batch Bpad: split-K
// weight-gradient partials and the bias-gradient partials' counts.
static AdamArgs step_args(mjp_surrogate* s, int Bpad) {
    AdamArgs a = adam_args(s);
    a.splits = wgrad_splits(s, Bpad);
    for (int l = 0; l < s->L; ++l) {
        a.lay[l].nbp = s->fused ? 1 : (l + 1 == s->L ? Bpad / kMseRows : Bpad / 64);
        if (s->fused) a.lay[l].bp = s->bgrad[l].as<float>();  // reduced by the weight-gradient launch
    }
    return a;
}

// loss partials one training step leaves at padded batch Bpad
static int loss_parts(const mjp_surrogate* s, int Bpad) { return s->fused ? Bpad / s->mt : Bpad / kMseRows; }

static FusedArgs fused_args(const mjp_surrogate* s, const float* x, const float* y, const int32_t* perm, int base,
                            int n_valid) {
    FusedArgs f{};
    f.L = s->L;
    f.width = s->cfg.width;
    f.in_dim = s->in[0];
    f.kpad0 = s->kpad[0];
    f.n_valid = n_valid;
    f.base = base;
    f.x = x;
    f.y = y;
    f.perm = perm;
    f.master = s->master.as<float>();
    for (int l = 0; l < s->L; ++l) {
        f.boff[l] = s->woff[l] + (int64_t)s->out[l] * s->in[l];
        f.W[l] = s->wbf[l].as<uint16_t>();
        f.WF[l] = s->wbfF[l].as<uint16_t>();
        f.WB[l] = s->wbfB[l].as<uint16_t>();
        f.X[l] = s->X[l].as<uint16_t>();
        f.dZ[l] = s->dZ[l].as<uint16_t>();
        f.bpart[l] = s->bpart[l].as<float>();
    }
    return f;
}

static hipError_t fused_lds_limits() {
    const void* fns[] = {reinterpret_cast<const void*>(k_mlp_fused<true, 1>),
                         reinterpret_cast<const void*>(k_mlp_fused<false, 1>)};
    hipError_t e = hipSuccess;
    for (const void* f : fns)
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_wgrad_all), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kGemmLds);
    return e;
}

// One fused training pass over rows base.. (forward, loss, backward data)
// into X, dZ, the bias partials and the loss partials lp, then every
// layer's weight-gradient partials.
static void fused_train_pass(mjp_surrogate* s, const float* x, const float* y, const int32_t* perm, int base,
                             int n_valid, int Bpad, double* lp, hipStream_t st) {
    static const hipError_t lds_ok = fused_lds_limits();  // a failure surfaces as a launch error
    (void)lds_ok;
    FusedArgs f = fused_args(s, x, y, perm, base, n_valid);
    f.lossp = lp;
    hipLaunchKernelGGL((k_mlp_fused<true, 1>), dim3(Bpad / 16), dim3(kFThreads),
                       fused_lds_bytes(true, s->L, s->cfg.width, 16), st, f);
    WgradAll w{};
    w.L = s->L;
    const int splits = wgrad_splits(s, Bpad);
    int blocks = 0;
    for (int l = 0; l < s->L; ++l) {
        GemmArgs& g = w.g[l];
        g.M = s->npad[l];
        g.N = s->kpad[l];
        g.K = Bpad;
        g.A = s->dZ[l].as<uint16_t>();
        g.lda = s->npad[l];
        g.B = s->X[l].as<uint16_t>();
        g.ldb = s->kpad[l];
        g.k_per_split = Bpad / splits;
        g.P = s->P[l].as<float>();
        w.start[l] = blocks;
        blocks += (g.N / kTN) * (g.M / kTM) * splits;
    }
    w.start[s->L] = blocks;
    int bb = 0;
    for (int l = 0; l < s->L; ++l) {
        w.bstart[l] = bb;
        w.bpart[l] = s->bpart[l].as<float>();
        w.bgrad[l] = s->bgrad[l].as<float>();
        bb += s->npad[l] / 64;
    }
    w.bstart[s->L] = bb;
    w.nbp = Bpad / s->mt;
    blocks += bb;
    hipLaunchKernelGGL(k_wgrad_all, dim3(blocks), dim3(kGT), kGemmLds, st, w);
}

}  // namespace mjp

extern "C" {

mjp_status mjp_surrogate_create(const mjp_mlp_cfg* cfg, uint64_t seed, mjp_surrogate** out) {
    clear_error();
    MJP_CHECK(out, MJP_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    MJP_CHECK(cfg, MJP_E_INVALID_ARG, "cfg is NULL");
    MJP_CHECK(cfg->in_dim >= 1 && cfg->in_dim <= 16, MJP_E_INVALID_ARG, "in_dim must be in [1, 16]");
    MJP_CHECK(cfg->width >= 64 && cfg->width <= 512 && cfg->width % 64 == 0, MJP_E_INVALID_ARG,
              "width must be a multiple of 64 in [64, 512]");
    MJP_CHECK(cfg->depth >= 1 && cfg->depth <= kMaxLayers - 1, MJP_E_INVALID_ARG, "depth must be in [1, %d]",
              kMaxLayers - 1);
    mjp_surrogate* s = new (std::nothrow) mjp_surrogate();
    MJP_CHECK(s, MJP_E_DEVICE, "out of host memory");
    s->cfg = *cfg;
    s->L = cfg->depth + 1;
    int64_t off = 0;
    for (int l = 0; l < s->L; ++l) {
        s->in[l] = l == 0 ? cfg->in_dim : cfg->width;
        s->out[l] = l + 1 == s->L ? 1 : cfg->width;
        s->kpad[l] = round_up(s->in[l], 64);
        s->npad[l] = round_up(s->out[l], 64);
        s->woff[l] = off;
        off += (int64_t)s->in[l] * s->out[l] + s->out[l];
    }
    s->woff[s->L] = off;
    s->total = off;
    // the fused step's rows per workgroup: 16 (32 halves the weight loads per row but
    // leaves half the CUs idle at batch 4096: 1.87% against 2.05% of the BF16 peak)
    s->mt = 16;
    s->fused = cfg->width <= kFMaxW && fused_lds_bytes(true, s->L, cfg->width, s->mt) <= 160 * 1024;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(MJP_E_DEVICE, "no HIP device available");
    }
    // PyTorch-style default init: U(-1/sqrt(in), 1/sqrt(in)) for weights and biases
    std::vector<float> h((size_t)s->total);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < s->L; ++l) {
        const float bound = 1.0f / std::sqrt((float)s->in[l]);
        std::uniform_real_distribution<float> U(-bound, bound);
        for (int64_t p = s->woff[l]; p < s->woff[l + 1]; ++p) h[(size_t)p] = U(rng);
    }
    mjp_status st;
    if ((st = s->master.reserve(sizeof(float) * s->total)) || (st = s->m1.reserve(sizeof(float) * s->total)) ||
        (st = s->m2.reserve(sizeof(float) * s->total))) {
        mjp_surrogate_destroy(s);
        return st;
    }
    for (int l = 0; l < s->L; ++l) {
        const size_t wb = sizeof(uint16_t) * (size_t)s->npad[l] * s->kpad[l];
        if ((st = s->wbf[l].reserve(wb)) || (st = s->wbfF[l].reserve(wb)) || (st = s->wbfB[l].reserve(wb))) {
            mjp_surrogate_destroy(s);
            return st;
        }
        if (hipMemset(s->wbf[l].ptr, 0, wb) != hipSuccess || hipMemset(s->wbfF[l].ptr, 0, wb) != hipSuccess ||
            hipMemset(s->wbfB[l].ptr, 0, wb) != hipSuccess) {
            mjp_surrogate_destroy(s);
            return fail(MJP_E_DEVICE, "hipMemset failed");
        }
    }
    if (hipMemcpy(s->master.ptr, h.data(), sizeof(float) * s->total, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->m1.ptr, 0, sizeof(float) * s->total) != hipSuccess ||
        hipMemset(s->m2.ptr, 0, sizeof(float) * s->total) != hipSuccess) {
        mjp_surrogate_destroy(s);
        return fail(MJP_E_DEVICE, "parameter upload failed");
    }
    AdamArgs a = adam_args(s);
    hipLaunchKernelGGL(k_refresh_bf16, dim3((unsigned)((s->total + 255) / 256)), dim3(256), 0, 0, a);
    if (hipDeviceSynchronize() != hipSuccess) {
        mjp_surrogate_destroy(s);
        return fail(MJP_E_DEVICE, "init kernel failed");
    }
    *out = s;
    return MJP_OK;
}

void mjp_surrogate_destroy(mjp_surrogate* s) {
    if (!s) return;
    s->master.release();
    s->m1.release();
    s->m2.release();
    s->gradbuf.release();
    for (int l = 0; l < kMaxLayers; ++l) {
        s->wbf[l].release();
        s->wbfF[l].release();
        s->wbfB[l].release();
        s->P[l].release();
        s->Z[l].release();
        s->dZ[l].release();
        s->bpart[l].release();
        s->bgrad[l].release();
    }
    for (auto& b : s->X) b.release();
    s->Y.release();
    s->tgt.release();
    s->lossp.release();
    s->perm.release();
    delete s;
}

int64_t mjp_surrogate_num_params(const mjp_surrogate* s) { return s ? s->total : 0; }

mjp_status mjp_surrogate_get_params(const mjp_surrogate* s, float* params_h, int64_t count) {
    clear_error();
    MJP_CHECK(s && params_h, MJP_E_INVALID_ARG, "null argument");
    MJP_CHECK(count == s->total, MJP_E_INVALID_ARG, "count %lld != %lld parameters", (long long)count,
              (long long)s->total);
    MJP_HIP(hipMemcpy(params_h, s->master.ptr, sizeof(float) * s->total, hipMemcpyDeviceToHost));
    return MJP_OK;
}

mjp_status mjp_surrogate_set_params(mjp_surrogate* s, const float* params_h, int64_t count) {
    clear_error();
    MJP_CHECK(s && params_h, MJP_E_INVALID_ARG, "null argument");
    MJP_CHECK(count == s->total, MJP_E_INVALID_ARG, "count %lld != %lld parameters", (long long)count,
              (long long)s->total);
    for (int64_t p = 0; p < count; ++p) MJP_CHECK(std::isfinite(params_h[p]), MJP_E_INVALID_ARG, "non-finite parameter");
    MJP_HIP(hipMemcpy(s->master.ptr, params_h, sizeof(float) * s->total, hipMemcpyHostToDevice));
    MJP_HIP(hipMemset(s->m1.ptr, 0, sizeof(float) * s->total));
    MJP_HIP(hipMemset(s->m2.ptr, 0, sizeof(float) * s->total));
    s->step = 0;
    AdamArgs a = adam_args(s);
    hipLaunchKernelGGL(k_refresh_bf16, dim3((unsigned)((s->total + 255) / 256)), dim3(256), 0, 0, a);
    MJP_HIP(hipDeviceSynchronize());
    return MJP_OK;
}

mjp_status mjp_surrogate_infer(const mjp_surrogate* sc, const float* x_d, int32_t n, float* y_d, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(sc, MJP_E_INVALID_ARG, "surrogate is NULL");
    MJP_CHECK(n >= 0, MJP_E_INVALID_ARG, "n must be >= 0");
    if (n == 0) return MJP_OK;
    MJP_CHECK(x_d && y_d, MJP_E_INVALID_ARG, "null buffer");
    mjp_surrogate* s = const_cast<mjp_surrogate*>(sc);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (s->fused) {  // one launch, no work buffers
        static const hipError_t lds_ok = fused_lds_limits();
        (void)lds_ok;
        FusedArgs f = fused_args(s, x_d, nullptr, nullptr, 0, n);
        f.yout = y_d;
        hipLaunchKernelGGL((k_mlp_fused<false, 1>), dim3((unsigned)((n + 15) / 16)), dim3(kFThreads),
                           fused_lds_bytes(false, s->L, s->cfg.width, 16), st, f);
        MJP_HIP(hipGetLastError());
        return MJP_OK;
    }
    const int chunk = 4096;
    mjp_status e = surrogate_alloc(s, std::max(s->Bmax, std::min(chunk, round_up(n, 256))), st);
    if (e) return e;
    for (int base = 0; base < n; base += s->Bmax) {
        const int nv = std::min(s->Bmax, n - base);
        const int Bpad = round_up(nv, 256);
        load_rows(s, x_d, nullptr, nullptr, base, nv, Bpad, st);
        forward(s, Bpad, nv, st);
        hipLaunchKernelGGL(k_copy_col0, dim3((nv + 255) / 256), dim3(256), 0, st, s->Y.as<float>(), s->npad[s->L - 1],
                           nv, y_d + base);
    }
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}

mjp_status mjp_surrogate_grad(const mjp_surrogate* sc, const float* x_d, const float* y_d, int32_t n, float* grad_h,
                              float* loss_h, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(sc && x_d && y_d && grad_h, MJP_E_INVALID_ARG, "null argument");
    MJP_CHECK(n >= 1 && n <= 65536, MJP_E_INVALID_ARG, "n must be in [1, 65536]");
    mjp_surrogate* s = const_cast<mjp_surrogate*>(sc);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int Bpad = round_up(n, 512);
    mjp_status e = surrogate_alloc(s, Bpad, st);
    if (e) return e;
    if ((e = s->gradbuf.reserve(sizeof(float) * s->total))) return e;
    if (s->fused) {
        fused_train_pass(s, x_d, y_d, nullptr, 0, n, Bpad, s->lossp.as<double>(), st);
    } else {
        load_rows(s, x_d, y_d, nullptr, 0, n, Bpad, st);
        forward(s, Bpad, n, st);
        loss_grad(s, n, Bpad, s->lossp.as<double>(), st);
        backward(s, Bpad, st);
    }
    AdamArgs a = step_args(s, Bpad);
    a.grad_out = s->gradbuf.as<float>();
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((s->total + 255) / 256)), dim3(256), 0, st, a);
    MJP_HIP(hipGetLastError());
    std::vector<double> lp((size_t)loss_parts(s, Bpad));
    MJP_HIP(hipMemcpyAsync(lp.data(), s->lossp.ptr, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, st));
    MJP_HIP(hipMemcpyAsync(grad_h, s->gradbuf.ptr, sizeof(float) * s->total, hipMemcpyDeviceToHost, st));
    MJP_HIP(hipStreamSynchronize(st));
    if (loss_h) {
        double tot = 0.0;
        for (double v : lp) tot += v;
        *loss_h = (float)(tot / n);
    }
    return MJP_OK;
}

mjp_status mjp_surrogate_train(mjp_surrogate* s, const float* x_d, const float* y_d, int32_t n,
                               const mjp_train_cfg* cfg, float* loss_h, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(s && x_d && y_d && cfg, MJP_E_INVALID_ARG, "null argument");
    MJP_CHECK(n >= 1, MJP_E_INVALID_ARG, "n must be >= 1");
    MJP_CHECK(cfg->epochs >= 1 && cfg->batch >= 512 && cfg->batch % 512 == 0 && cfg->batch <= 65536,
              MJP_E_INVALID_ARG, "epochs >= 1 and batch a multiple of 512 in [512, 65536]");
    MJP_CHECK(std::isfinite(cfg->lr) && cfg->lr > 0 && cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 &&
                  cfg->beta2 < 1 && cfg->eps_adam > 0 && cfg->weight_decay >= 0,
              MJP_E_INVALID_ARG, "bad optimiser settings");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mjp_status e = surrogate_alloc(s, cfg->batch, st);
    if (e) return e;
    // The host runs ahead of the device: no step waits for the previous one.
    // Each epoch's permutation goes to one of two device slots from one of
    // two pinned host buffers (copied by a kernel on the stream), reused once
    // the epoch two back has finished (an event per slot, recorded after the
    // epoch's last step); the loss partials of every step stay on the
    // device and are read once at the end.
    const int nb = (n + cfg->batch - 1) / cfg->batch;
    const int lstride = loss_parts(s, cfg->batch);  // loss partials per step
    if ((e = s->perm.reserve(sizeof(int32_t) * 2 * (size_t)n))) return e;
    if (loss_h && (e = s->lossp.reserve(sizeof(double) * (size_t)cfg->epochs * nb * lstride))) return e;
    int32_t* ph[2] = {nullptr, nullptr};
    int32_t* ph_d[2] = {nullptr, nullptr};  // device addresses of the pinned slots
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto cleanup = [&]() {
        for (int q = 0; q < 2; ++q) {
            if (ev[q]) (void)hipEventDestroy(ev[q]);
            if (ph[q]) (void)hipHostFree(ph[q]);
        }
    };
    for (int q = 0; q < 2; ++q) {
        if (hipHostMalloc(reinterpret_cast<void**>(&ph[q]), sizeof(int32_t) * (size_t)n,
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
            hipHostGetDevicePointer(reinterpret_cast<void**>(&ph_d[q]), ph[q], 0) != hipSuccess ||
            hipEventCreateWithFlags(&ev[q], hipEventDisableTiming) != hipSuccess) {
            cleanup();
            return fail(MJP_E_DEVICE, "pinned permutation buffers or events could not be created");
        }
    }
    std::mt19937_64 rng(cfg->seed);
    hipError_t he = hipSuccess;
    for (int ep = 0; ep < cfg->epochs && he == hipSuccess; ++ep) {
        const int slot = ep & 1;
        if (ep >= 2 && (he = hipEventSynchronize(ev[slot])) != hipSuccess) break;  // epoch ep - 2 is done with it
        int32_t* perm = ph[slot];
        for (int i = 0; i < n; ++i) perm[i] = i;
        std::shuffle(perm, perm + n, rng);
        int32_t* perm_d = s->perm.as<int32_t>() + (size_t)slot * n;
        hipLaunchKernelGGL(k_copy_perm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ph_d[slot], perm_d, n);
        for (int bi = 0; bi < nb; ++bi) {
            const int base = bi * cfg->batch;
            const int nv = std::min(cfg->batch, n - base);
            const int Bpad = round_up(nv, 512);
            double* lp = loss_h ? s->lossp.as<double>() + ((size_t)ep * nb + bi) * lstride : s->lossp.as<double>();
            if (s->fused) {
                fused_train_pass(s, x_d, y_d, perm_d, base, nv, Bpad, lp, st);
            } else {
                load_rows(s, x_d, y_d, perm_d, base, nv, Bpad, st);
                forward(s, Bpad, nv, st);
                loss_grad(s, nv, Bpad, lp, st);
                backward(s, Bpad, st);
            }
            s->step += 1;
            AdamArgs a = step_args(s, Bpad);
            a.lr = cfg->lr;
            a.beta1 = cfg->beta1;
            a.beta2 = cfg->beta2;
            a.eps = cfg->eps_adam;
            a.wd = cfg->weight_decay;
            a.bc1 = 1.f - std::pow(cfg->beta1, (float)s->step);
            a.bc2 = 1.f - std::pow(cfg->beta2, (float)s->step);
            hipLaunchKernelGGL(k_adam, dim3((unsigned)((s->total + 255) / 256)), dim3(256), 0, st, a);
        }
        if ((he = hipEventRecord(ev[slot], st)) != hipSuccess) break;
    }
    if (he == hipSuccess) he = hipGetLastError();
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    cleanup();
    MJP_CHECK(he == hipSuccess, MJP_E_DEVICE, "training failed: %s", hipGetErrorString(he));
    if (loss_h) {
        std::vector<double> lp((size_t)cfg->epochs * nb * lstride);
        MJP_HIP(hipMemcpy(lp.data(), s->lossp.ptr, sizeof(double) * lp.size(), hipMemcpyDeviceToHost));
        for (int ep = 0; ep < cfg->epochs; ++ep) {
            double ep_loss = 0.0;
            for (int bi = 0; bi < nb; ++bi) {
                const int nv = std::min(cfg->batch, n - bi * cfg->batch);
                const int used = loss_parts(s, round_up(nv, 512));
                for (int c = 0; c < used; ++c) ep_loss += lp[((size_t)ep * nb + bi) * lstride + c];
            }
            loss_h[ep] = (float)(ep_loss / n);
        }
    }
    return MJP_OK;
}

mjp_status mjp_surrogate_save(const mjp_surrogate* s, const char* path) {
    clear_error();
    MJP_CHECK(s && path, MJP_E_INVALID_ARG, "null argument");
    std::vector<float> h((size_t)s->total);
    MJP_HIP(hipMemcpy(h.data(), s->master.ptr, sizeof(float) * s->total, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    MJP_CHECK(f, MJP_E_INVALID_ARG, "cannot open %s", path);
    const char magic[4] = {'M', 'J', 'P', 'S'};
    const int32_t hdr[4] = {1, s->cfg.in_dim, s->cfg.width, s->cfg.depth};
    const int64_t cnt = s->total;
    bool ok = std::fwrite(magic, 1, 4, f) == 4 && std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
              std::fwrite(&cnt, sizeof cnt, 1, f) == 1 && std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    MJP_CHECK(ok, MJP_E_INVALID_ARG, "write to %s failed", path);
    return MJP_OK;
}

mjp_status mjp_surrogate_load(const char* path, mjp_surrogate** out) {
    clear_error();
    MJP_CHECK(path && out, MJP_E_INVALID_ARG, "null argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    MJP_CHECK(f, MJP_E_INVALID_ARG, "cannot open %s", path);
    char magic[4];
    int32_t hdr[4];
    int64_t cnt = 0;
    bool ok = std::fread(magic, 1, 4, f) == 4 && std::memcmp(magic, "MJPS", 4) == 0 &&
              std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 1 && std::fread(&cnt, sizeof cnt, 1, f) == 1 &&
              cnt > 0 && cnt < ((int64_t)1 << 28);
    std::vector<float> h;
    if (ok) {
        h.resize((size_t)cnt);
        ok = std::fread(h.data(), sizeof(float), h.size(), f) == h.size();
    }
    std::fclose(f);
    MJP_CHECK(ok, MJP_E_INVALID_ARG, "%s is not a surrogate file", path);
    mjp_mlp_cfg cfg{hdr[1], hdr[2], hdr[3]};
    mjp_surrogate* s = nullptr;
    mjp_status st = mjp_surrogate_create(&cfg, 0, &s);
    if (st) return st;
    if (cnt != s->total) {
        mjp_surrogate_destroy(s);
        return fail(MJP_E_INVALID_ARG, "%s: parameter count does not match its configuration", path);
    }
    if ((st = mjp_surrogate_set_params(s, h.data(), cnt))) {
        mjp_surrogate_destroy(s);
        return st;
    }
    *out = s;
    return MJP_OK;
}

}  // extern "C"
