// Metropolis-Hastings and delayed-acceptance chains on the device.
//
// Random walk in log-rates psi = log(theta) with the prior Normal(mu, sigma)
// on every log-rate (SI: sampling scheme and prior); the exact
// log-likelihood of every scored proposal is the R-MJP expansion (Sec.
// 2.1.2, the batched likelihood kernels).  Delayed acceptance (Christen and
// Fox, J. Comput. Graph. Stat. 14(4), 2005): a screen -- the MLP surrogate of
// the log-likelihood plus the exact log-prior -- accepts or rejects first
// with probability min(1, exp(s(psi') - s(psi))); only the proposals it
// accepts are scored exactly, and a second test with min(1, exp((l(psi') -
// l(psi)) - (s(psi') - s(psi)))) keeps the exact posterior invariant.
//
// One step is a fixed sequence of launches on one stream, with no host read:
//   k_smp_propose   Philox4x32-10 draws, proposal psi' = psi + L z, theta' =
//                   exp(psi'), the screen's standardised input
//   (DA) surrogate inference on every chain's proposal
//   k_smp_screen    stage 1 (DA) and the mask of proposals to score
//   likelihood      the masked batched log-likelihood (loglik_run)
//   k_smp_accept    stage 2 (DA) or the MH test; state update, sample row,
//                   counters; the step counter advances
// so a step (or several) can be captured in a hipGraph and replayed: the
// random numbers are a function of (seed, chain, step counter), the sample
// row is the step counter modulo the caller's ring of rows.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter and a
// 64-bit key, ten rounds of two 32x32->64-bit multiplications by the round
// constants with the halves exchanged and xored with the counter words and
// the key, the key bumped by the Weyl constants between rounds.  Counter of
// chain c at step h, block q: (c, h mod 2^32, h / 2^32, q); blocks 0..2 give
// up to six normals (Box-Muller on pairs of 53-bit uniforms), block 3 the
// two acceptance uniforms.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace mjp {

constexpr int kSmpMaxPar = 6;
constexpr int kSmpBlock = 256;
constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

__host__ __device__ inline void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// uniform in (0, 1] from two words (53 bits)
__host__ __device__ inline double u53(uint32_t a, uint32_t b) {
    const double x = ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
    return 1.0 - x;
}

struct SmpArgs {
    double* psi;          // [C][d] current states
    double* lp;           // [C] exact log-posterior of the states
    double* sc;           // [C] screened log-posterior of the states (DA)
    double* prop;         // [C][d] proposals
    double* theta;        // [C][stride] exp(proposal), zero-padded
    float* x;             // [C][d] standardised proposals (screen input)
    const float* y;       // [C] screen output (standardised log-likelihood)
    double* scp;          // [C] screened log-posterior of the proposals
    double* u;            // [C][2] acceptance uniforms
    const double* ll;     // [C] exact log-likelihood of the proposals
    uint8_t* active;      // [C] proposals to score exactly
    unsigned long long* ctr;  // [4] step, accepted, stage-1 accepted, exact evaluations
    double* samples;      // [ring][C][d] or null
    int32_t ring;
    int32_t C, d, stride;
    int32_t da;           // 1: delayed acceptance
    uint32_t key[2];
    double L[kSmpMaxPar * kSmpMaxPar];  // Cholesky factor of the proposal covariance, row-major
    double smean[kSmpMaxPar], sstd[kSmpMaxPar];
    double ll_mean, ll_std;
    double prior_mu, prior_sigma;
};

__device__ inline double log_prior(const double* p, int d, double mu, double sigma) {
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
        const double z = (p[j] - mu) / sigma;
        s += -0.5 * z * z;
    }
    return s;
}

__device__ inline unsigned long long wave_count(bool v) {
    return (unsigned long long)__popcll(__ballot(v));
}

__global__ __launch_bounds__(kSmpBlock) void k_smp_propose(SmpArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    const unsigned long long h = a.ctr[0];
    double z[kSmpMaxPar];
    uint32_t r[4];
    for (int q = 0; q < 3; ++q) {
        const uint32_t cw[4] = {(uint32_t)c, (uint32_t)h, (uint32_t)(h >> 32), (uint32_t)q};
        philox4x32_10(cw, a.key, r);
        const double u1 = u53(r[0], r[1]), u2 = u53(r[2], r[3]);
        const double rad = sqrt(-2.0 * log(u1)), ang = 6.283185307179586 * u2;
        if (2 * q < kSmpMaxPar) z[2 * q] = rad * cos(ang);
        if (2 * q + 1 < kSmpMaxPar) z[2 * q + 1] = rad * sin(ang);
    }
    {
        const uint32_t cw[4] = {(uint32_t)c, (uint32_t)h, (uint32_t)(h >> 32), 3u};
        philox4x32_10(cw, a.key, r);
        a.u[2 * c] = u53(r[0], r[1]);
        a.u[2 * c + 1] = u53(r[2], r[3]);
    }
    const double* p = a.psi + (size_t)c * a.d;
    double* q = a.prop + (size_t)c * a.d;
    double* th = a.theta + (size_t)c * a.stride;
    for (int j = 0; j < a.stride; ++j) th[j] = 0.0;
    for (int j = 0; j < a.d; ++j) {
        double v = p[j];
        for (int k = 0; k <= j; ++k) v += a.L[j * kSmpMaxPar + k] * z[k];
        q[j] = v;
        th[j] = exp(v);
        if (a.da) a.x[(size_t)c * a.d + j] = (float)((v - a.smean[j]) / a.sstd[j]);
    }
}

// stage 1 (DA) and the mask of proposals the likelihood scores
__global__ __launch_bounds__(kSmpBlock) void k_smp_screen(SmpArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    bool act = false;
    if (c < a.C) {
        if (a.da) {
            const double s = (double)a.y[c] * a.ll_std + a.ll_mean +
                             log_prior(a.prop + (size_t)c * a.d, a.d, a.prior_mu, a.prior_sigma);
            a.scp[c] = s;
            act = log(a.u[2 * c]) < s - a.sc[c];
        } else {
            act = true;
        }
        a.active[c] = act ? 1 : 0;
    }
    const unsigned long long n = wave_count(act);
    if ((threadIdx.x & 63) == 0 && n) {
        atomicAdd(a.ctr + 3, n);
        if (a.da) atomicAdd(a.ctr + 2, n);
    }
}

__global__ __launch_bounds__(kSmpBlock) void k_smp_accept(SmpArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    bool acc = false;
    if (c < a.C) {
        double* p = a.psi + (size_t)c * a.d;
        if (a.active[c]) {
            const double* q = a.prop + (size_t)c * a.d;
            const double lpp = a.ll[c] + log_prior(q, a.d, a.prior_mu, a.prior_sigma);
            double thr = lpp - a.lp[c];
            if (a.da) thr -= a.scp[c] - a.sc[c];
            acc = lpp > -INFINITY && log(a.u[2 * c + 1]) < thr;  // NaN and -inf reject
            if (acc) {
                for (int j = 0; j < a.d; ++j) p[j] = q[j];
                a.lp[c] = lpp;
                if (a.da) a.sc[c] = a.scp[c];
            }
        }
        if (a.samples) {
            const unsigned long long h = a.ctr[0];
            double* row = a.samples + ((size_t)(h % (unsigned long long)a.ring) * a.C + c) * a.d;
            for (int j = 0; j < a.d; ++j) row[j] = p[j];
        }
    }
    const unsigned long long n = wave_count(acc);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(a.ctr + 1, n);
}

// after every chain has read the step counter
__global__ void k_smp_advance(unsigned long long* ctr) { ctr[0] += 1ull; }

// initial states: theta = exp(psi) for the likelihood, the screen's input
__global__ __launch_bounds__(kSmpBlock) void k_smp_init_inputs(SmpArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    const double* p = a.psi + (size_t)c * a.d;
    double* th = a.theta + (size_t)c * a.stride;
    for (int j = 0; j < a.stride; ++j) th[j] = 0.0;
    for (int j = 0; j < a.d; ++j) {
        th[j] = exp(p[j]);
        if (a.da) a.x[(size_t)c * a.d + j] = (float)((p[j] - a.smean[j]) / a.sstd[j]);
    }
}

__global__ __launch_bounds__(kSmpBlock) void k_smp_init_post(SmpArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    const double lpr = log_prior(a.psi + (size_t)c * a.d, a.d, a.prior_mu, a.prior_sigma);
    a.lp[c] = a.ll[c] + lpr;
    if (a.da) a.sc[c] = (double)a.y[c] * a.ll_std + a.ll_mean + lpr;
}

__global__ void k_smp_set_counters(unsigned long long* ctr, unsigned long long s0, unsigned long long s1,
                                   unsigned long long s2, unsigned long long s3) {
    ctr[0] = s0;
    ctr[1] = s1;
    ctr[2] = s2;
    ctr[3] = s3;
}

__global__ void k_philox_fill(uint32_t key0, uint32_t key1, uint32_t c1, uint32_t c2, uint32_t c3, int32_t n,
                              uint32_t* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t cw[4] = {(uint32_t)i, c1, c2, c3}, key[2] = {key0, key1};
    uint32_t r[4];
    philox4x32_10(cw, key, r);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = r[j];
}

// ---------------------------------------------------------------- J-MJP
// Poisson(lambda) from counter (c0, c1, c2, attempt).  lambda < 10:
// inversion of the cumulative distribution (one uniform, the terms built by
// the ratio lambda / k).  lambda >= 10: the transformed rejection method
// with squeeze of Hoermann ("The transformed rejection method for generating
// Poisson random variables", Insurance: Mathematics and Economics 12, 1993):
// a candidate k = floor((2a/us + b) U + lambda + 0.43) from U uniform on
// (-1/2, 1/2), us = 1/2 - |U|, accepted at once inside the squeeze (us >=
// 0.07, V <= v_r) and otherwise by comparing log(V alpha^-1 / (a/us^2 + b))
// with the log-pmf; a fresh attempt counter per candidate.
constexpr int kPoisAttempts = 64;  // each attempt is accepted with probability > 0.85

__host__ __device__ inline int32_t poisson_draw(double lam, const uint32_t key[2], uint32_t c0, uint32_t c1,
                                                uint32_t c2) {
    if (!(lam > 0.0)) return 0;
    uint32_t r[4];
    if (lam < 10.0) {
        const uint32_t cw[4] = {c0, c1, c2, 0u};
        philox4x32_10(cw, key, r);
        const double u = 1.0 - u53(r[0], r[1]);  // [0, 1)
        double p = exp(-lam), F = p;
        int32_t k = 0;
        while (u >= F && k < 1000) {
            ++k;
            p *= lam / (double)k;
            F += p;
        }
        return k;
    }
    const double slam = sqrt(lam), loglam = log(lam);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    const double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (uint32_t at = 0; at < (uint32_t)kPoisAttempts; ++at) {
        const uint32_t cw[4] = {c0, c1, c2, at};
        philox4x32_10(cw, key, r);
        const double U = u53(r[0], r[1]) - 0.5, V = u53(r[2], r[3]);
        const double us = 0.5 - fabs(U);
        const double k = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return (int32_t)k;
        if (k < 0.0 || (us < 0.013 && V > us)) continue;
        if (log(V) + log(invalpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1.0))
            return (int32_t)k;
    }
    return (int32_t)floor(lam);  // not reached in practice (probability < 1e-50)
}

// log Poisson(k | W)
__device__ inline double log_poisson(int32_t k, double W) {
    if (W > 0.0) return (double)k * log(W) - W - lgamma((double)k + 1.0);
    return k == 0 ? 0.0 : -INFINITY;
}

constexpr uint32_t kJmTheta = 0xFFFFFFFFu;  // observation word of the theta draws
constexpr uint32_t kJmKAcc = 100u;          // attempt word of a jump count's acceptance uniform
constexpr uint32_t kJmBurn = 0x80000000u;   // step word of the jump-count burn-in sweeps
constexpr uint32_t kJmInit = 0xFFFFFFFEu;   // step word of the initial jump counts

struct JmArgs {
    double* psi;      // [C][d]
    double* prop;     // [C][d]
    double* theta;    // [C][stride] exp of the states (k sweep) or of the proposals
    int32_t* k;       // [C][I]
    int32_t* kprop;   // [C][I]
    double* logphi;   // [C][I] log p(s_i | k_i, theta)
    double* lpp;      // [C][I] the same at the proposal
    double* omega;    // [C]
    double* omp;      // [C]
    double* lt;       // [C] log target of the states
    const double* Tobs;  // [I]
    unsigned long long* ctr;  // [4] steps, theta accepted, jump counts accepted, jump counts proposed
    double* samples;
    int32_t ring, C, I, d, stride;
    uint32_t key[2];
    double L[kSmpMaxPar * kSmpMaxPar];
    double prior_mu, prior_sigma;
};

__global__ __launch_bounds__(kSmpBlock) void k_jm_theta_of_states(JmArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    double* th = a.theta + (size_t)c * a.stride;
    for (int j = 0; j < a.stride; ++j) th[j] = j < a.d ? exp(a.psi[(size_t)c * a.d + j]) : 0.0;
}

// k'_ci ~ Poisson(Omega_c T_i); step word h (or kJmInit: the initial counts, written to k)
__global__ __launch_bounds__(kSmpBlock) void k_jm_kprop(JmArgs a, uint32_t hword, int to_k) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.C * a.I) return;
    const int c = (int)(idx / a.I), i = (int)(idx - (int64_t)c * a.I);
    const uint32_t h = hword == 0u ? (uint32_t)a.ctr[0] : hword;
    const int32_t kk = poisson_draw(a.omega[c] * a.Tobs[i], a.key, (uint32_t)c, (uint32_t)i, h);
    (to_k ? a.k : a.kprop)[idx] = kk;
}

// accept each proposed jump count with min(1, phi(k') / phi(k)) (the
// proposal is the jump-count prior, which cancels)
__global__ __launch_bounds__(kSmpBlock) void k_jm_kaccept(JmArgs a, uint32_t hword) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool acc = false;
    if (idx < (int64_t)a.C * a.I) {
        const int c = (int)(idx / a.I), i = (int)(idx - (int64_t)c * a.I);
        const uint32_t h = hword == 0u ? (uint32_t)a.ctr[0] : hword;
        const uint32_t cw[4] = {(uint32_t)c, (uint32_t)i, h, kJmKAcc};
        uint32_t r[4];
        philox4x32_10(cw, a.key, r);
        acc = log(u53(r[0], r[1])) < a.lpp[idx] - a.logphi[idx];
        if (acc) {
            a.k[idx] = a.kprop[idx];
            a.logphi[idx] = a.lpp[idx];
        }
    }
    const unsigned long long n = wave_count(acc);
    const unsigned long long m = wave_count(idx < (int64_t)a.C * a.I);
    if ((threadIdx.x & 63) == 0) {
        if (n) atomicAdd(a.ctr + 2, n);
        if (m) atomicAdd(a.ctr + 3, m);
    }
}

__global__ __launch_bounds__(kSmpBlock) void k_jm_propose(JmArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    const uint32_t h = (uint32_t)a.ctr[0];
    double z[kSmpMaxPar];
    uint32_t r[4];
    for (int q = 0; q < 3; ++q) {
        const uint32_t cw[4] = {(uint32_t)c, kJmTheta, h, (uint32_t)q};
        philox4x32_10(cw, a.key, r);
        const double u1 = u53(r[0], r[1]), u2 = u53(r[2], r[3]);
        const double rad = sqrt(-2.0 * log(u1)), ang = 6.283185307179586 * u2;
        if (2 * q < kSmpMaxPar) z[2 * q] = rad * cos(ang);
        if (2 * q + 1 < kSmpMaxPar) z[2 * q + 1] = rad * sin(ang);
    }
    const double* p = a.psi + (size_t)c * a.d;
    double* q = a.prop + (size_t)c * a.d;
    double* th = a.theta + (size_t)c * a.stride;
    for (int j = 0; j < a.stride; ++j) th[j] = 0.0;
    for (int j = 0; j < a.d; ++j) {
        double v = p[j];
        for (int k = 0; k <= j; ++k) v += a.L[j * kSmpMaxPar + k] * z[k];
        q[j] = v;
        th[j] = exp(v);
    }
}

__device__ inline double block_sum_256(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kSmpBlock / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// one workgroup per chain: log target sum_i [log Poisson(k_i | Omega T_i) +
// log phi_i] + log prior.  mode 0: of the states (lt); mode 1: of the
// proposal, then the Metropolis test on theta and the state update.
__global__ __launch_bounds__(kSmpBlock) void k_jm_target(JmArgs a, int mode) {
    __shared__ double red[kSmpBlock / 64];
    const int c = blockIdx.x;
    const double om = mode ? a.omp[c] : a.omega[c];
    const double* phi = (mode ? a.lpp : a.logphi) + (size_t)c * a.I;
    const int32_t* kk = a.k + (size_t)c * a.I;
    double v = 0.0;
    for (int i = threadIdx.x; i < a.I; i += kSmpBlock) v += log_poisson(kk[i], om * a.Tobs[i]) + phi[i];
    const double tot = block_sum_256(v, red) +
                       log_prior((mode ? a.prop : a.psi) + (size_t)c * a.d, a.d, a.prior_mu, a.prior_sigma);
    if (!mode) {
        if (threadIdx.x == 0) a.lt[c] = tot;
        return;
    }
    const uint32_t h = (uint32_t)a.ctr[0];
    const uint32_t cw[4] = {(uint32_t)c, kJmTheta, h, 3u};
    uint32_t r[4];
    philox4x32_10(cw, a.key, r);
    const bool acc = tot > -INFINITY && log(u53(r[0], r[1])) < tot - a.lt[c];
    if (acc) {
        for (int i = threadIdx.x; i < a.I; i += kSmpBlock) a.logphi[(size_t)c * a.I + i] = phi[i];
        if (threadIdx.x < a.d) a.psi[(size_t)c * a.d + threadIdx.x] = a.prop[(size_t)c * a.d + threadIdx.x];
        if (threadIdx.x == 0) {
            a.omega[c] = om;
            a.lt[c] = tot;
            atomicAdd(a.ctr + 1, 1ull);
        }
    }
    if (a.samples) {
        __syncthreads();
        double* row = a.samples + ((size_t)(a.ctr[0] % (unsigned long long)a.ring) * a.C + c) * a.d;
        if (threadIdx.x < a.d) row[threadIdx.x] = a.psi[(size_t)c * a.d + threadIdx.x];
    }
}

__global__ void k_poisson_fill(uint32_t key0, uint32_t key1, uint32_t c1, const double* lam, int32_t n, int32_t* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t key[2] = {key0, key1};
    out[i] = poisson_draw(lam[i], key, (uint32_t)i, c1, 0u);
}

}  // namespace mjp

using namespace mjp;

struct mjp_sampler {
    int device = 0;
    mjp_sampler_cfg cfg{};
    mjp_opts opts{};
    int d = 0, stride = 4;
    std::vector<double> T;
    std::vector<int32_t> rec;
    mjp_obs obs{};
    double L[kSmpMaxPar * kSmpMaxPar] = {};
    const mjp_surrogate* screen = nullptr;
    double smean[kSmpMaxPar] = {}, sstd[kSmpMaxPar] = {};
    double ll_mean = 0.0, ll_std = 1.0;
    bool has_state = false;
    DevBuf psi, lp, sc, prop, theta, x, y, scp, u, ll, active, ctr, dims;
};

struct mjp_jmjp {
    int device = 0;
    mjp_sampler_cfg cfg{};
    mjp_opts opts{};
    int d = 0, stride = 4, I = 0;
    std::vector<double> T;
    std::vector<int32_t> rec;
    mjp_obs obs{};
    double L[kSmpMaxPar * kSmpMaxPar] = {};
    bool has_state = false;
    DevBuf psi, prop, theta, k, kprop, logphi, lpp, omega, omp, lt, Tobs, ctr, dims;
};

static JmArgs jm_args(const mjp_jmjp* s, double* samples, int ring) {
    JmArgs a{};
    a.psi = s->psi.as<double>();
    a.prop = s->prop.as<double>();
    a.theta = s->theta.as<double>();
    a.k = s->k.as<int32_t>();
    a.kprop = s->kprop.as<int32_t>();
    a.logphi = s->logphi.as<double>();
    a.lpp = s->lpp.as<double>();
    a.omega = s->omega.as<double>();
    a.omp = s->omp.as<double>();
    a.lt = s->lt.as<double>();
    a.Tobs = s->Tobs.as<double>();
    a.ctr = s->ctr.as<unsigned long long>();
    a.samples = samples;
    a.ring = ring > 0 ? ring : 1;
    a.C = s->cfg.chains;
    a.I = s->I;
    a.d = s->d;
    a.stride = s->stride;
    a.key[0] = (uint32_t)s->cfg.seed;
    a.key[1] = (uint32_t)(s->cfg.seed >> 32);
    std::memcpy(a.L, s->L, sizeof a.L);
    a.prior_mu = s->cfg.prior_mu;
    a.prior_sigma = s->cfg.prior_sigma;
    return a;
}

__global__ void k_jm_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static SmpArgs smp_args(const mjp_sampler* s, bool da, double* samples, int ring) {
    SmpArgs a{};
    a.psi = s->psi.as<double>();
    a.lp = s->lp.as<double>();
    a.sc = s->sc.as<double>();
    a.prop = s->prop.as<double>();
    a.theta = s->theta.as<double>();
    a.x = s->x.as<float>();
    a.y = s->y.as<float>();
    a.scp = s->scp.as<double>();
    a.u = s->u.as<double>();
    a.ll = s->ll.as<double>();
    a.active = s->active.as<uint8_t>();
    a.ctr = s->ctr.as<unsigned long long>();
    a.samples = samples;
    a.ring = ring > 0 ? ring : 1;
    a.C = s->cfg.chains;
    a.d = s->d;
    a.stride = s->stride;
    a.da = da ? 1 : 0;
    a.key[0] = (uint32_t)s->cfg.seed;
    a.key[1] = (uint32_t)(s->cfg.seed >> 32);
    std::memcpy(a.L, s->L, sizeof a.L);
    std::memcpy(a.smean, s->smean, sizeof a.smean);
    std::memcpy(a.sstd, s->sstd, sizeof a.sstd);
    a.ll_mean = s->ll_mean;
    a.ll_std = s->ll_std;
    a.prior_mu = s->cfg.prior_mu;
    a.prior_sigma = s->cfg.prior_sigma;
    return a;
}

struct SmpGuard {  // the sampler's device for the call's duration
    int prev = -1;
    explicit SmpGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~SmpGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

extern "C" {

void mjp_sampler_cfg_default(mjp_sampler_cfg* c) {
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->model = MJP_MODEL_CASCADE2;
    c->chains = 256;
    c->seed = 1;
    c->prior_mu = 1.0;
    c->prior_sigma = 1e5;
}

mjp_status mjp_sampler_create(const mjp_sampler_cfg* cfg, const mjp_obs* obs, const mjp_opts* opts,
                              mjp_sampler** out) {
    clear_error();
    MJP_CHECK(cfg && obs && opts && out, MJP_E_INVALID_ARG, "null argument");
    *out = nullptr;
    MJP_CHECK(cfg->model >= MJP_MODEL_BD && cfg->model <= MJP_MODEL_AUTOREG, MJP_E_INVALID_ARG, "unknown model %d",
              cfg->model);
    const int npar = cfg->model == MJP_MODEL_BD ? 2 : (cfg->model == MJP_MODEL_AUTOREG ? 6 : 4);
    MJP_CHECK(cfg->chains >= 1 && cfg->chains <= (1 << 24), MJP_E_INVALID_ARG, "chains must be in [1, 2^24]");
    MJP_CHECK(cfg->dims[0] >= 1 && (cfg->model == MJP_MODEL_BD || cfg->dims[1] >= 1), MJP_E_INVALID_ARG,
              "bad grid (%d, %d)", cfg->dims[0], cfg->dims[1]);
    MJP_CHECK(std::isfinite(cfg->prior_mu) && cfg->prior_sigma > 0.0 && std::isfinite(cfg->prior_sigma),
              MJP_E_INVALID_ARG, "prior needs a finite mean and a positive finite sigma");
    MJP_CHECK(obs->n_t >= 1 && obs->T_h && obs->n_obs >= 1 && obs->obs_h, MJP_E_INVALID_ARG, "empty observations");
    mjp_sampler* s = new (std::nothrow) mjp_sampler();
    MJP_CHECK(s, MJP_E_DEVICE, "out of host memory");
    s->cfg = *cfg;
    s->opts = *opts;
    s->d = npar;
    s->stride = cfg->model == MJP_MODEL_AUTOREG ? 6 : 4;
    s->T.assign(obs->T_h, obs->T_h + obs->n_t);
    s->rec.assign(obs->obs_h, obs->obs_h + 4 * (size_t)obs->n_obs);
    s->obs = *obs;
    s->obs.T_h = s->T.data();
    s->obs.obs_h = s->rec.data();
    for (int j = 0; j < kSmpMaxPar; ++j) s->sstd[j] = 1.0;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(MJP_E_DEVICE, "no device");
    }
    const size_t C = (size_t)cfg->chains, d = (size_t)npar;
    mjp_status st;
    if ((st = s->psi.reserve(sizeof(double) * C * d)) || (st = s->lp.reserve(sizeof(double) * C)) ||
        (st = s->sc.reserve(sizeof(double) * C)) || (st = s->prop.reserve(sizeof(double) * C * d)) ||
        (st = s->theta.reserve(sizeof(double) * C * (size_t)s->stride)) || (st = s->x.reserve(sizeof(float) * C * d)) ||
        (st = s->y.reserve(sizeof(float) * C)) || (st = s->scp.reserve(sizeof(double) * C)) ||
        (st = s->u.reserve(sizeof(double) * 2 * C)) || (st = s->ll.reserve(sizeof(double) * C)) ||
        (st = s->active.reserve(C)) || (st = s->ctr.reserve(sizeof(unsigned long long) * 4)) ||
        (st = s->dims.reserve(sizeof(int32_t) * 2 * C))) {
        mjp_sampler_destroy(s);
        return st;
    }
    std::vector<int32_t> dm(2 * C);
    for (size_t c = 0; c < C; ++c) {
        dm[2 * c] = cfg->dims[0];
        dm[2 * c + 1] = cfg->model == MJP_MODEL_BD ? 1 : cfg->dims[1];
    }
    if (hipMemcpy(s->dims.ptr, dm.data(), sizeof(int32_t) * dm.size(), hipMemcpyHostToDevice) != hipSuccess) {
        mjp_sampler_destroy(s);
        return fail(MJP_E_DEVICE, "hipMemcpy failed");
    }
    *out = s;
    return MJP_OK;
}

void mjp_sampler_destroy(mjp_sampler* s) {
    if (!s) return;
    SmpGuard g(s->device);
    for (DevBuf* b : {&s->psi, &s->lp, &s->sc, &s->prop, &s->theta, &s->x, &s->y, &s->scp, &s->u, &s->ll, &s->active,
                      &s->ctr, &s->dims})
        b->release();
    delete s;
}

mjp_status mjp_sampler_set_proposal(mjp_sampler* s, const double* chol_h) {
    clear_error();
    MJP_CHECK(s && chol_h, MJP_E_INVALID_ARG, "null argument");
    const int d = s->d;
    double L[kSmpMaxPar * kSmpMaxPar] = {};
    for (int i = 0; i < d; ++i)
        for (int k = 0; k < d; ++k) {
            const double v = chol_h[i * d + k];
            MJP_CHECK(std::isfinite(v), MJP_E_INVALID_ARG, "non-finite factor entry (%d, %d)", i, k);
            MJP_CHECK(k <= i || v == 0.0, MJP_E_INVALID_ARG, "the factor must be lower triangular");
            L[i * kSmpMaxPar + k] = v;
        }
    std::memcpy(s->L, L, sizeof L);
    return MJP_OK;
}

mjp_status mjp_sampler_set_screen(mjp_sampler* s, const mjp_surrogate* screen, const double* psi_mean_h,
                                  const double* psi_std_h, double ll_mean, double ll_std) {
    clear_error();
    MJP_CHECK(s, MJP_E_INVALID_ARG, "null sampler");
    if (!screen) {
        s->screen = nullptr;
        return MJP_OK;
    }
    MJP_CHECK(psi_mean_h && psi_std_h, MJP_E_INVALID_ARG, "null standardisation");
    MJP_CHECK(std::isfinite(ll_mean) && ll_std > 0.0 && std::isfinite(ll_std), MJP_E_INVALID_ARG,
              "bad output scale");
    for (int j = 0; j < s->d; ++j)
        MJP_CHECK(std::isfinite(psi_mean_h[j]) && psi_std_h[j] > 0.0 && std::isfinite(psi_std_h[j]),
                  MJP_E_INVALID_ARG, "bad input scale %d", j);
    s->screen = screen;
    for (int j = 0; j < s->d; ++j) {
        s->smean[j] = psi_mean_h[j];
        s->sstd[j] = psi_std_h[j];
    }
    s->ll_mean = ll_mean;
    s->ll_std = ll_std;
    return MJP_OK;
}

mjp_status mjp_sampler_init(mjp_sampler* s, const double* psi0_d, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(s && psi0_d, MJP_E_INVALID_ARG, "null argument");
    SmpGuard g(s->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int C = s->cfg.chains;
    MJP_HIP(hipMemcpyAsync(s->psi.ptr, psi0_d, sizeof(double) * (size_t)C * s->d, hipMemcpyDeviceToDevice, st));
    const bool da = s->screen != nullptr;
    const SmpArgs a = smp_args(s, da, nullptr, 1);
    const unsigned grid = (unsigned)((C + kSmpBlock - 1) / kSmpBlock);
    hipLaunchKernelGGL(k_smp_init_inputs, dim3(grid), dim3(kSmpBlock), 0, st, a);
    hipLaunchKernelGGL(k_smp_set_counters, dim3(1), dim3(1), 0, st, a.ctr, 0ull, 0ull, 0ull, 0ull);
    mjp_status r = loglik_run(s->cfg.model, C, s->theta.as<double>(), s->dims.as<int32_t>(), &s->obs, &s->opts,
                              nullptr, s->ll.as<double>(), nullptr, st);
    if (r) return r;
    if (da && (r = mjp_surrogate_infer(s->screen, s->x.as<float>(), C, s->y.as<float>(), stream))) return r;
    hipLaunchKernelGGL(k_smp_init_post, dim3(grid), dim3(kSmpBlock), 0, st, a);
    MJP_HIP(hipGetLastError());
    s->has_state = true;
    return MJP_OK;
}

mjp_status mjp_sampler_run(mjp_sampler* s, int32_t steps, double* samples_d, int32_t ring_rows, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(s, MJP_E_INVALID_ARG, "null sampler");
    MJP_CHECK(steps >= 0, MJP_E_INVALID_ARG, "steps must be >= 0");
    MJP_CHECK(!samples_d || ring_rows >= 1, MJP_E_INVALID_ARG, "ring_rows must be >= 1 with a sample array");
    MJP_CHECK(s->has_state, MJP_E_INVALID_ARG, "no state: call mjp_sampler_init or mjp_sampler_set_state first");
    SmpGuard g(s->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int C = s->cfg.chains;
    const bool da = s->screen != nullptr;
    const SmpArgs a = smp_args(s, da, samples_d, ring_rows);
    const unsigned grid = (unsigned)((C + kSmpBlock - 1) / kSmpBlock);
    for (int32_t h = 0; h < steps; ++h) {
        hipLaunchKernelGGL(k_smp_propose, dim3(grid), dim3(kSmpBlock), 0, st, a);
        mjp_status r;
        if (da && (r = mjp_surrogate_infer(s->screen, s->x.as<float>(), C, s->y.as<float>(), stream))) return r;
        hipLaunchKernelGGL(k_smp_screen, dim3(grid), dim3(kSmpBlock), 0, st, a);
        if ((r = loglik_run(s->cfg.model, C, s->theta.as<double>(), s->dims.as<int32_t>(), &s->obs, &s->opts,
                            da ? s->active.as<uint8_t>() : nullptr, s->ll.as<double>(), nullptr, st)))
            return r;
        hipLaunchKernelGGL(k_smp_accept, dim3(grid), dim3(kSmpBlock), 0, st, a);
        hipLaunchKernelGGL(k_smp_advance, dim3(1), dim3(1), 0, st, a.ctr);
    }
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}

mjp_status mjp_sampler_get_state(const mjp_sampler* s, double* psi_h, double* lp_h, double* sc_h, uint64_t* counters_h,
                                 mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(s && psi_h && lp_h && sc_h && counters_h, MJP_E_INVALID_ARG, "null argument");
    MJP_CHECK(s->has_state, MJP_E_INVALID_ARG, "no state yet");
    SmpGuard g(s->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t C = (size_t)s->cfg.chains;
    MJP_HIP(hipMemcpyAsync(psi_h, s->psi.ptr, sizeof(double) * C * s->d, hipMemcpyDeviceToHost, st));
    MJP_HIP(hipMemcpyAsync(lp_h, s->lp.ptr, sizeof(double) * C, hipMemcpyDeviceToHost, st));
    MJP_HIP(hipMemcpyAsync(sc_h, s->sc.ptr, sizeof(double) * C, hipMemcpyDeviceToHost, st));
    MJP_HIP(hipMemcpyAsync(counters_h, s->ctr.ptr, sizeof(uint64_t) * 4, hipMemcpyDeviceToHost, st));
    MJP_HIP(hipStreamSynchronize(st));
    return MJP_OK;
}

mjp_status mjp_sampler_set_state(mjp_sampler* s, const double* psi_h, const double* lp_h, const double* sc_h,
                                 const uint64_t* counters_h, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(s && psi_h && lp_h && sc_h && counters_h, MJP_E_INVALID_ARG, "null argument");
    SmpGuard g(s->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t C = (size_t)s->cfg.chains;
    MJP_HIP(hipMemcpyAsync(s->psi.ptr, psi_h, sizeof(double) * C * s->d, hipMemcpyHostToDevice, st));
    MJP_HIP(hipMemcpyAsync(s->lp.ptr, lp_h, sizeof(double) * C, hipMemcpyHostToDevice, st));
    MJP_HIP(hipMemcpyAsync(s->sc.ptr, sc_h, sizeof(double) * C, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_smp_set_counters, dim3(1), dim3(1), 0, st, s->ctr.as<unsigned long long>(),
                       (unsigned long long)counters_h[0], (unsigned long long)counters_h[1],
                       (unsigned long long)counters_h[2], (unsigned long long)counters_h[3]);
    MJP_HIP(hipStreamSynchronize(st));
    s->has_state = true;
    return MJP_OK;
}

mjp_status mjp_philox_fill(uint64_t key, uint32_t c1, uint32_t c2, uint32_t c3, int32_t n, uint32_t* out_d,
                           mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(n >= 0 && (n == 0 || out_d), MJP_E_INVALID_ARG, "bad output");
    if (n == 0) return MJP_OK;
    hipLaunchKernelGGL(k_philox_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), (uint32_t)key, (uint32_t)(key >> 32), c1, c2, c3, n,
                       out_d);
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}

void mjp_philox4x32_10(const uint32_t* ctr4, const uint32_t* key2, uint32_t* out4) {
    if (!ctr4 || !key2 || !out4) return;
    philox4x32_10(ctr4, key2, out4);
}

mjp_status mjp_poisson_fill(uint64_t key, uint32_t c1, const double* lam_d, int32_t n, int32_t* out_d,
                            mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(n >= 0 && (n == 0 || (lam_d && out_d)), MJP_E_INVALID_ARG, "bad arrays");
    if (n == 0) return MJP_OK;
    hipLaunchKernelGGL(k_poisson_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), (uint32_t)key, (uint32_t)(key >> 32), c1, lam_d, n,
                       out_d);
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}

// ---- J-MJP Gibbs chains
mjp_status mjp_jmjp_create(const mjp_sampler_cfg* cfg, const mjp_obs* obs, const mjp_opts* opts, mjp_jmjp** out) {
    clear_error();
    MJP_CHECK(cfg && obs && opts && out, MJP_E_INVALID_ARG, "null argument");
    *out = nullptr;
    MJP_CHECK(cfg->model >= MJP_MODEL_BD && cfg->model <= MJP_MODEL_AUTOREG, MJP_E_INVALID_ARG, "unknown model %d",
              cfg->model);
    MJP_CHECK(cfg->chains >= 1 && cfg->chains <= (1 << 24), MJP_E_INVALID_ARG, "chains must be in [1, 2^24]");
    MJP_CHECK(cfg->dims[0] >= 1 && (cfg->model == MJP_MODEL_BD || cfg->dims[1] >= 1), MJP_E_INVALID_ARG,
              "bad grid (%d, %d)", cfg->dims[0], cfg->dims[1]);
    MJP_CHECK(std::isfinite(cfg->prior_mu) && cfg->prior_sigma > 0.0 && std::isfinite(cfg->prior_sigma),
              MJP_E_INVALID_ARG, "prior needs a finite mean and a positive finite sigma");
    MJP_CHECK(obs->n_t >= 1 && obs->T_h && obs->n_obs >= 1 && obs->obs_h, MJP_E_INVALID_ARG, "empty observations");
    for (int32_t i = 0; i < obs->n_obs; ++i) {
        MJP_CHECK(obs->obs_h[4 * i + 3] == 1, MJP_E_INVALID_ARG, "record %d: each observation has its own jump count",
                  i);
        MJP_CHECK(obs->obs_h[4 * i] >= 0 && obs->obs_h[4 * i] < obs->n_t, MJP_E_INVALID_ARG, "record %d: bad time", i);
    }
    mjp_jmjp* s = new (std::nothrow) mjp_jmjp();
    MJP_CHECK(s, MJP_E_DEVICE, "out of host memory");
    s->cfg = *cfg;
    s->opts = *opts;
    s->d = cfg->model == MJP_MODEL_BD ? 2 : (cfg->model == MJP_MODEL_AUTOREG ? 6 : 4);
    s->stride = cfg->model == MJP_MODEL_AUTOREG ? 6 : 4;
    s->I = obs->n_obs;
    s->T.assign(obs->T_h, obs->T_h + obs->n_t);
    s->rec.assign(obs->obs_h, obs->obs_h + 4 * (size_t)obs->n_obs);
    s->obs = *obs;
    s->obs.T_h = s->T.data();
    s->obs.obs_h = s->rec.data();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(MJP_E_DEVICE, "no device");
    }
    const size_t C = (size_t)cfg->chains, d = (size_t)s->d, I = (size_t)s->I;
    mjp_status st;
    if ((st = s->psi.reserve(sizeof(double) * C * d)) || (st = s->prop.reserve(sizeof(double) * C * d)) ||
        (st = s->theta.reserve(sizeof(double) * C * (size_t)s->stride)) || (st = s->k.reserve(sizeof(int32_t) * C * I)) ||
        (st = s->kprop.reserve(sizeof(int32_t) * C * I)) || (st = s->logphi.reserve(sizeof(double) * C * I)) ||
        (st = s->lpp.reserve(sizeof(double) * C * I)) || (st = s->omega.reserve(sizeof(double) * C)) ||
        (st = s->omp.reserve(sizeof(double) * C)) || (st = s->lt.reserve(sizeof(double) * C)) ||
        (st = s->Tobs.reserve(sizeof(double) * I)) || (st = s->ctr.reserve(sizeof(unsigned long long) * 4)) ||
        (st = s->dims.reserve(sizeof(int32_t) * 2 * C))) {
        mjp_jmjp_destroy(s);
        return st;
    }
    std::vector<int32_t> dm(2 * C);
    for (size_t c = 0; c < C; ++c) {
        dm[2 * c] = cfg->dims[0];
        dm[2 * c + 1] = cfg->model == MJP_MODEL_BD ? 1 : cfg->dims[1];
    }
    std::vector<double> To(I);
    for (size_t i = 0; i < I; ++i) To[i] = s->T[(size_t)s->rec[4 * i]];
    if (hipMemcpy(s->dims.ptr, dm.data(), sizeof(int32_t) * dm.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->Tobs.ptr, To.data(), sizeof(double) * I, hipMemcpyHostToDevice) != hipSuccess) {
        mjp_jmjp_destroy(s);
        return fail(MJP_E_DEVICE, "hipMemcpy failed");
    }
    *out = s;
    return MJP_OK;
}

void mjp_jmjp_destroy(mjp_jmjp* s) {
    if (!s) return;
    SmpGuard g(s->device);
    for (DevBuf* b : {&s->psi, &s->prop, &s->theta, &s->k, &s->kprop, &s->logphi, &s->lpp, &s->omega, &s->omp, &s->lt,
                      &s->Tobs, &s->ctr, &s->dims})
        b->release();
    delete s;
}

mjp_status mjp_jmjp_set_proposal(mjp_jmjp* s, const double* chol_h) {
    clear_error();
    MJP_CHECK(s && chol_h, MJP_E_INVALID_ARG, "null argument");
    double L[kSmpMaxPar * kSmpMaxPar] = {};
    for (int i = 0; i < s->d; ++i)
        for (int k = 0; k < s->d; ++k) {
            const double v = chol_h[i * s->d + k];
            MJP_CHECK(std::isfinite(v), MJP_E_INVALID_ARG, "non-finite factor entry (%d, %d)", i, k);
            MJP_CHECK(k <= i || v == 0.0, MJP_E_INVALID_ARG, "the factor must be lower triangular");
            L[i * kSmpMaxPar + k] = v;
        }
    std::memcpy(s->L, L, sizeof L);
    return MJP_OK;
}

// the jump counts' probabilities at the states' theta for counts kbuf
static mjp_status jm_probs(mjp_jmjp* s, const int32_t* kbuf, double* out, double* om, hipStream_t st) {
    return mjp_jump_probs(s->cfg.model, s->cfg.chains, s->theta.as<double>(), s->dims.as<int32_t>(), &s->obs, kbuf,
                          &s->opts, out, om, reinterpret_cast<mjp_stream_t>(st));
}

mjp_status mjp_jmjp_init(mjp_jmjp* s, const double* psi0_d, int32_t k_burn, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(s && psi0_d, MJP_E_INVALID_ARG, "null argument");
    MJP_CHECK(k_burn >= 0 && k_burn < (1 << 30), MJP_E_INVALID_ARG, "k_burn out of range");
    SmpGuard g(s->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int C = s->cfg.chains;
    const int64_t CI = (int64_t)C * s->I;
    MJP_HIP(hipMemcpyAsync(s->psi.ptr, psi0_d, sizeof(double) * (size_t)C * s->d, hipMemcpyDeviceToDevice, st));
    const JmArgs a = jm_args(s, nullptr, 1);
    const unsigned gc = (unsigned)((C + kSmpBlock - 1) / kSmpBlock), gi = (unsigned)((CI + kSmpBlock - 1) / kSmpBlock);
    hipLaunchKernelGGL(k_smp_set_counters, dim3(1), dim3(1), 0, st, a.ctr, 0ull, 0ull, 0ull, 0ull);
    hipLaunchKernelGGL(k_jm_theta_of_states, dim3(gc), dim3(kSmpBlock), 0, st, a);
    // Omega at the start (jump counts 0), then counts from their prior
    hipLaunchKernelGGL(k_jm_fill_i32, dim3(gi), dim3(kSmpBlock), 0, st, a.k, CI, 0);
    mjp_status r;
    if ((r = jm_probs(s, a.k, a.logphi, a.omega, st))) return r;
    hipLaunchKernelGGL(k_jm_kprop, dim3(gi), dim3(kSmpBlock), 0, st, a, kJmInit, 1);
    if ((r = jm_probs(s, a.k, a.logphi, a.omega, st))) return r;
    for (int32_t j = 0; j < k_burn; ++j) {
        hipLaunchKernelGGL(k_jm_kprop, dim3(gi), dim3(kSmpBlock), 0, st, a, kJmBurn + (uint32_t)j, 0);
        if ((r = jm_probs(s, a.kprop, a.lpp, a.omp, st))) return r;
        hipLaunchKernelGGL(k_jm_kaccept, dim3(gi), dim3(kSmpBlock), 0, st, a, kJmBurn + (uint32_t)j);
    }
    hipLaunchKernelGGL(k_jm_target, dim3((unsigned)C), dim3(kSmpBlock), 0, st, a, 0);
    hipLaunchKernelGGL(k_smp_set_counters, dim3(1), dim3(1), 0, st, a.ctr, 0ull, 0ull, 0ull, 0ull);
    MJP_HIP(hipGetLastError());
    s->has_state = true;
    return MJP_OK;
}

mjp_status mjp_jmjp_run(mjp_jmjp* s, int32_t steps, double* samples_d, int32_t ring_rows, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(s, MJP_E_INVALID_ARG, "null chains");
    MJP_CHECK(steps >= 0, MJP_E_INVALID_ARG, "steps must be >= 0");
    MJP_CHECK(!samples_d || ring_rows >= 1, MJP_E_INVALID_ARG, "ring_rows must be >= 1 with a sample array");
    MJP_CHECK(s->has_state, MJP_E_INVALID_ARG, "call mjp_jmjp_init first");
    SmpGuard g(s->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int C = s->cfg.chains;
    const int64_t CI = (int64_t)C * s->I;
    const JmArgs a = jm_args(s, samples_d, ring_rows);
    const unsigned gc = (unsigned)((C + kSmpBlock - 1) / kSmpBlock), gi = (unsigned)((CI + kSmpBlock - 1) / kSmpBlock);
    for (int32_t h = 0; h < steps; ++h) {
        mjp_status r;
        // every jump count given theta (Eq. sam_k), then theta given the counts (Eq. sam_th)
        hipLaunchKernelGGL(k_jm_theta_of_states, dim3(gc), dim3(kSmpBlock), 0, st, a);
        hipLaunchKernelGGL(k_jm_kprop, dim3(gi), dim3(kSmpBlock), 0, st, a, 0u, 0);
        if ((r = jm_probs(s, a.kprop, a.lpp, a.omp, st))) return r;
        hipLaunchKernelGGL(k_jm_kaccept, dim3(gi), dim3(kSmpBlock), 0, st, a, 0u);
        hipLaunchKernelGGL(k_jm_propose, dim3(gc), dim3(kSmpBlock), 0, st, a);
        if ((r = jm_probs(s, a.k, a.lpp, a.omp, st))) return r;
        hipLaunchKernelGGL(k_jm_target, dim3((unsigned)C), dim3(kSmpBlock), 0, st, a, 1);
        hipLaunchKernelGGL(k_smp_advance, dim3(1), dim3(1), 0, st, a.ctr);
    }
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}

mjp_status mjp_jmjp_counters(const mjp_jmjp* s, uint64_t* counters_h, mjp_stream_t stream) {
    clear_error();
    MJP_CHECK(s && counters_h, MJP_E_INVALID_ARG, "null argument");
    SmpGuard g(s->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    MJP_HIP(hipMemcpyAsync(counters_h, s->ctr.ptr, sizeof(uint64_t) * 4, hipMemcpyDeviceToHost, st));
    MJP_HIP(hipStreamSynchronize(st));
    return MJP_OK;
}

}  // extern "C"
