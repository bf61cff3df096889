// Persistent R-MJP sweep: all K jumps, the weighted accumulation and the
// lumping in ONE cooperative launch.
//
// Layout: workgroup g (after an XCD-aware renumbering so each XCD owns a
// contiguous band of rows) owns WAVES*R consecutive 64-row slices; lane l of
// wave w holds rows slice*64 + l of its R slices.  For a CSR plan each
// thread loads its rows' entries of B^T (column, value) into registers once,
// so the operator is read from memory once per solve instead of once per jump.
// For a stencil plan each thread keeps its rows' five coefficients in
// registers.  The Kahan pairs (s, c) of the open collection windows live in
// registers too.  Per jump only the iterate moves: each thread gathers x at
// its columns and writes its rows of y.
//
// Jumps are separated by neighbour synchronisation (per-workgroup epoch
// flags) or, every renorm_every jumps and for operators without a narrow
// interval, a two-level grid barrier.  Every poll loop is bounded: on
// timeout the workgroup raises a flag and leaves the loop, so the kernel
// always ends.
//
// Two memory protocols make y of jump k visible to every XCD before jump k+1
// reads it:
//  * COH (default): the iterate is read and written only with device-scope
//    (agent) relaxed atomic loads and stores, which the hardware performs at
//    the device coherence point (the sc1 cache policy), never leaving a
//    dirty or stale copy in an XCD's L2.  Each wave waits for its own
//    stores to complete (s_waitcnt vmcnt(0)) before the workgroup publishes
//    its flag; a reader issues its loads only after it has seen the flag.
//    This keeps exactly the two hardware facts that the compiler's own
//    agent-scope release/acquire mapping rests on (a device-scope store is
//    visible device-wide once its counter has drained; a device-scope load
//    reads the coherent value), and drops the per-workgroup L2 write-back
//    and invalidate, which only plain (non-atomic) accesses need.  Those two
//    cache operations, issued by all ~32 workgroups of an XCD every jump,
//    cost more than the jump's data movement.
//  * fenced: plain loads and stores of the iterate, published with the
//    compiler's agent-scope release fence and consumed after an agent-scope
//    acquire fence (L2 write-back / invalidate).  Kept as the reference
//    protocol; both protocols give bit-identical results.
#include <algorithm>
#include <unordered_map>
#include <array>
#include <climits>
#include <cstring>
#include <cmath>
#include <vector>

#include "gridsync.h"
#include "internal.h"
#include "sweep.h"

namespace mjp {

constexpr int kPWaves = 8;            // waves per workgroup
constexpr int kPThreads = 64 * kPWaves;
constexpr int kPSlots = 4;            // open collection windows held in registers
constexpr uint8_t kSliceLocal = 1;   // per-slice table bit (see build_sweep_tables)

struct PersistArgs {
    const int32_t* __restrict__ slice_off;
    const int32_t* __restrict__ col;
    const float* __restrict__ val;
    const float* __restrict__ dlo;    // CSR: lo part of each row's diagonal (entry 0 holds hi)
    StencilCoef cf;
    const float* __restrict__ rho0;
    float* __restrict__ buf0;
    float* __restrict__ buf1;
    float* __restrict__ out;
    const double* __restrict__ wtab;
    double* __restrict__ pmass;   // [3][G] FP64 partial masses (initial, renorm double buffer)
    unsigned* __restrict__ bar;   // [kBarWords] barrier words, zero at launch
    unsigned* __restrict__ wflag; // [G * 32] per-workgroup epoch flags (one 128-byte line each), zero at launch
    const int32_t* __restrict__ wait;  // [G][2] neighbour interval [lo, hi] or null (global barriers only)
    const uint8_t* __restrict__ sflag; // [n_slices] kSliceLocal or 0
    const int32_t* __restrict__ p2;    // two-jump kernel: [G][kP2Tab] regions and neighbour interval
    unsigned* __restrict__ flags;
    double* __restrict__ mass_out;  // [2]: initial mass, last measured mass
    double* __restrict__ out_mass;  // item sweep only: FP64 mass of each output row, or null
    uint64_t timeout_ticks;         // per-barrier wait limit in wall-clock ticks
    int64_t n;
    int32_t n_slices;
    int32_t Kmax;
    int32_t renorm_every;
    int32_t G;
    AllTimes at;
    int32_t slot[kMaxTimes];
};

// Neighbour synchronisation after jump k: publish "my rows of step k are
// written" (publishing step + relaxed store of k to my flag line), then wait
// until every workgroup in my interval [lo, hi] has published k.  The
// interval covers the workgroups whose rows I read (their y of step k must
// be visible before I compute step k+1) and those that read my rows (they
// must have finished reading the buffer I overwrite at step k+1).  Lanes of
// wave 0 poll one flag each; in the fenced protocol the wave then issues one
// acquire fence.
template <bool COH, bool FORCE = false>
__device__ __forceinline__ bool neighbour_sync(unsigned* wflag, int lo, int hi, unsigned k, int g,
                                               unsigned* flags, uint64_t timeout_ticks) {
    __shared__ int aborted;
    drain_wave<COH>();
    __syncthreads();
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        if (lane == 0) {
            aborted = 0;
            release_agent<COH>();
            __hip_atomic_store(&wflag[g * 32], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const int h = lo + lane;
        bool bad = false;
        if (h <= hi && h != g) {
            if constexpr (FORCE) {  // give up at the first unready read (see gridsync.h)
                if (__hip_atomic_load(&wflag[h * 32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
                    __hip_atomic_fetch_or(flags, kFlagBarrierTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bad = true;
                }
            } else {
                const uint64_t t0 = wall_clock64();
                unsigned spins = 0;
                while (__hip_atomic_load(&wflag[h * 32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins % kAbortCheckEvery != 0) continue;
                    if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagBarrierTimeout) {
                        bad = true;
                        break;
                    }
                    if (wall_clock64() - t0 > timeout_ticks) {
                        __hip_atomic_fetch_or(flags, kFlagBarrierTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        bad = true;
                        break;
                    }
                }
            }
        }
        acquire_agent<COH>();
        if (bad) aborted = 1;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(aborted) == 0;  // uniform: every thread read the same word
}

// neighbour_sync over an explicit set: lane l < nn of wave 0 waits for
// workgroup nb[l] (the tiled sweep: the workgroups whose rows I read and
// those that read mine, eight for an interior tile).
__device__ __forceinline__ bool neighbour_sync_set(unsigned* wflag, const int32_t* nb, int nn, unsigned k, int g,
                                                   unsigned* flags, uint64_t timeout_ticks) {
    __shared__ int aborted;
    drain_wave<true>();
    __syncthreads();
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        if (lane == 0) {
            aborted = 0;
            __hip_atomic_store(&wflag[g * 32], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        bool bad = false;
        if (lane < nn) {
            const int h = nb[lane];
            const uint64_t t0 = wall_clock64();
            unsigned spins = 0;
            while (__hip_atomic_load(&wflag[h * 32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins % kAbortCheckEvery != 0) continue;
                if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagBarrierTimeout) {
                    bad = true;
                    break;
                }
                if (wall_clock64() - t0 > timeout_ticks) {
                    __hip_atomic_fetch_or(flags, kFlagBarrierTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

__device__ __forceinline__ double block_sum_f64(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kPWaves; ++i) s += red[i];
    __syncthreads();
    return s;  // valid in thread 0
}

// Sum of the G partials in a fixed order (identical in every workgroup).
__device__ __forceinline__ double sum_partials(const double* p, int G, double* red) {
    double v = 0.0;
    for (int i = threadIdx.x; i < G; i += kPThreads)
        v += __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double s = block_sum_f64(v, red);
    if (threadIdx.x == 0) red[kPWaves] = s;
    __syncthreads();
    s = red[kPWaves];
    __syncthreads();
    return s;
}

// The sweep of one workgroup's rows.  ITEMS: the single-workgroup form run
// once per item of a batch (G = 1; the whole vector is in LDS, so every
// gather is local and no slice table is read).
template <int R, int W, bool CSR, bool COH, bool ITEMS>
__device__ __forceinline__ void persistent_body(const PersistArgs& a) {
    __shared__ double red[kPWaves + 1];
    const int G = ITEMS ? 1 : a.G;
    const int g = ITEMS ? 0 : logical_block(G);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slice0 = (g * kPWaves + wave) * R;
    const int64_t n = a.n;

    // rows of this thread: row0 + 64 i, i < R (computed where used, which
    // keeps R registers free for the operator)
    const int32_t row0 = slice0 * 64 + lane;
    auto row = [&](int i) { return row0 + 64 * i; };
    auto live = [&](int i) { return (int64_t)(row0 + 64 * i) < n; };

    // ---- operator into registers
    // column of each entry, held as a 32-bit byte offset into the iterate so
    // each gather is a 32-bit register offset on a uniform base (n < 2^30).
    // Entry 0 is the diagonal (hi part; lo in dlo): its column is the row
    // itself, whose previous value the thread already holds, so coff[i][0]
    // is never read.
    uint32_t coff[R][W];
    float cval[R][W];
    float dlo[R];
    if (CSR) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int s = slice0 + i;
            int beg = 0, w = 0;
            if (s < a.n_slices) {
                beg = a.slice_off[s];
                w = (a.slice_off[s + 1] - beg) >> 6;
            }
#pragma unroll
            for (int j = 0; j < W; ++j) {
                if (live(i) && j < w) {
                    coff[i][j] = 4u * (uint32_t)a.col[beg + j * 64 + lane];
                    cval[i][j] = a.val[beg + j * 64 + lane];
                } else {
                    coff[i][j] = live(i) ? 4u * (uint32_t)row(i) : 0u;
                    cval[i][j] = 0.f;
                }
            }
            dlo[i] = live(i) ? a.dlo[row(i)] : 0.f;
        }
    } else {
        // stencil: each row's entries from the model (stencil_entries: the
        // diagonal first, then the inflows); absent entries get weight 0
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int64_t m = live(i) ? (int64_t)row(i) : 0;
            int32_t cc[W];
            float vv[W], lo;
            stencil_entries<W>(a.cf, m, cc, vv, lo);
            dlo[i] = live(i) ? lo : 0.f;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                coff[i][j] = 4u * (uint32_t)cc[j];
                cval[i][j] = live(i) ? vv[j] : 0.f;
            }
        }
    }

    // ---- this workgroup's rows of the iterate, double-buffered in LDS
    // Workgroup g owns rows [r0, r0 + kPWaves*R*64).  Slice i of a wave is
    // "local" when every column of every entry of its 64 rows is one of those
    // rows; a local slice gathers from the LDS copy (written by this
    // workgroup, visible after its own barrier), any other slice from the
    // iterate in global memory.  Every slice stores its rows to both.  The
    // bit is uniform per slice and fixed for the whole sweep (host-built
    // table).
    constexpr int kRowsWG = kPWaves * R * 64;
    __shared__ float ybuf[2][kRowsWG];
    const uint32_t lbase = 4u * (uint32_t)(g * kRowsWG);
    uint32_t lmask = 0;  // bit i: slice i is local
#pragma unroll
    for (int i = 0; i < R; ++i) {
        if (!live(i)) {
#pragma unroll
            for (int j = 0; j < W; ++j) coff[i][j] = lbase;  // padding lanes read a local row, weight 0
        }
        if constexpr (ITEMS) {
            lmask |= 1u << i;
        } else {
            const int sl = slice0 + i;
            const uint8_t f = sl < a.n_slices ? a.sflag[sl] : kSliceLocal;
            if (f & kSliceLocal) lmask |= 1u << i;
        }
    }
    lmask = __builtin_amdgcn_readfirstlane(lmask);
    const int lrow0 = wave * R * 64 + lane;  // this thread's row i sits at lrow0 + 64 i

    // ---- k = 0
    float sacc[kPSlots][R], cacc[kPSlots][R];
#pragma unroll
    for (int q = 0; q < kPSlots; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) { sacc[q][i] = 0.f; cacc[q][i] = 0.f; }

    float yv[R];
    double mloc = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        yv[i] = live(i) ? a.rho0[row(i)] : 0.f;
        if (live(i)) {
            if (!(yv[i] >= 0.f)) atomicOr(a.flags, (yv[i] != yv[i]) ? (unsigned)MJP_FLAG_NAN : (unsigned)MJP_FLAG_NEG);
            else if (isinf(yv[i])) atomicOr(a.flags, (unsigned)MJP_FLAG_NAN);
        }
        mloc += (double)yv[i];
        ybuf[0][lrow0 + 64 * i] = yv[i];
    }

    // Per-slot parameters of jump k (uniform): jq[q] is the time whose
    // window holds k in slot q (or -1), jL/jK/jO its window and output row.
    // They change only where a window opens or closes, so fetch() rescans
    // the kernel arguments only when k reaches knext, the first such jump
    // after the last scan.  The Poisson weights are held 64 jumps at a time: lane
    // l of wvec[q] is the weight of jump wbase + l for the time occupying
    // slot q then (0 if none), refilled every 64 jumps with one vector load
    // per lane, so a jump reads its weight from a register (v_readlane at a
    // uniform index) and never waits on memory for it.
    int jq[kPSlots], jL[kPSlots], jK[kPSlots], jO[kPSlots];
    int knext = 0;
    float wvec[kPSlots];
    int wbase = 0;
    auto fetch = [&](int k) {
        if (k >= knext) {
            knext = INT_MAX;
#pragma unroll
            for (int qq = 0; qq < kPSlots; ++qq) {
                jq[qq] = -1;
                jL[qq] = jK[qq] = jO[qq] = 0;
            }
            for (int j = 0; j < a.at.n; ++j) {
                const TimeParam& tp = a.at.tp[j];
                const int L = tp.L, K = tp.K;
                if (k < L) {
                    knext = min(knext, L);
                    continue;
                }
                if (k > K) continue;
                knext = min(knext, K + 1);
                const int o = tp.out, sj = a.slot[j];
#pragma unroll
                for (int qq = 0; qq < kPSlots; ++qq)
                    if (qq == sj) { jq[qq] = j; jL[qq] = L; jK[qq] = K; jO[qq] = o; }
            }
        }
        if ((k & 63) == 0) {
            wbase = k;
            const int kk = k + lane;
#pragma unroll
            for (int qq = 0; qq < kPSlots; ++qq) wvec[qq] = 0.f;
            for (int j = 0; j < a.at.n; ++j) {
                const TimeParam& tp = a.at.tp[j];
                if (kk < tp.L || kk > tp.K) continue;
                const float w = (kk == tp.K) ? (float)tp.lastw : (float)a.wtab[tp.woff + (kk - tp.L)];
#pragma unroll
                for (int qq = 0; qq < kPSlots; ++qq)
                    if (qq == a.slot[j]) wvec[qq] = w;
            }
        }
    };
    auto accumulate = [&](int k) {
#pragma unroll
        for (int qq = 0; qq < kPSlots; ++qq) {
            if (jq[qq] < 0) continue;
            const float w = __builtin_bit_cast(
                float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wvec[qq]), k - wbase));
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (k == jL[qq]) {
                    sacc[qq][i] = w * yv[i];
                    cacc[qq][i] = 0.f;
                } else {
                    const float yk = fmaf(w, yv[i], -cacc[qq][i]);
                    const float t = sacc[qq][i] + yk;
                    cacc[qq][i] = (t - sacc[qq][i]) - yk;
                    sacc[qq][i] = t;
                }
                if (k == jK[qq] && live(i)) a.out[(int64_t)jO[qq] * n + row(i)] = sacc[qq][i] - cacc[qq][i];
            }
            if constexpr (ITEMS) {
                if (k == jK[qq] && a.out_mass) {  // uniform: the row's mass for the item's report
                    double ms = 0.0;
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (live(i)) ms += (double)(sacc[qq][i] - cacc[qq][i]);
                    ms = block_sum_f64(ms, red);
                    if (threadIdx.x == 0) a.out_mass[jO[qq]] = ms;
                }
            }
        }
    };
    fetch(0);
    accumulate(0);

    // initial mass, reduced once all partials are in
    {
        const double s = block_sum_f64(mloc, red);
        if (threadIdx.x == 0) __hip_atomic_store(a.pmass + g, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned epoch = 1;
    if (!grid_barrier<COH>(a.bar, epoch, g, G, a.flags, a.timeout_ticks)) return;
    const double mass0 = sum_partials(a.pmass, G, red);
    double scale = 1.0;
    double last_mass = mass0;

    const int m = a.renorm_every;
    // renormalisation every m jumps (m = 0: never): rc counts down to the
    // next one, rpar is the parity of the renormalisations so far (selects
    // which of the two partial-mass arrays it writes)
    int rc = m, rpar = 0;
    // this workgroup's neighbour interval, read once
    const int wlo = a.wait ? a.wait[2 * g] : g, whi = a.wait ? a.wait[2 * g + 1] : g;
    const __amdgpu_buffer_rsrc_t r_rho0 = iter_rsrc(a.rho0, n), r_buf0 = iter_rsrc(a.buf0, n),
                                 r_buf1 = iter_rsrc(a.buf1, n);
    for (int k = 1; k <= a.Kmax; ++k) {
        const __amdgpu_buffer_rsrc_t x = (k == 1) ? r_rho0 : ((k & 1) ? r_buf0 : r_buf1);
        const __amdgpu_buffer_rsrc_t y = (k & 1) ? r_buf1 : r_buf0;
        const float fs = (float)scale;
        double part = 0.0;
        fetch(k);
        // all R*W gathers first, in one basic block, so they are in flight
        // together; the predicated stores come after every load was issued
        const char* __restrict__ xl = reinterpret_cast<const char*>(ybuf[(k - 1) & 1]) - lbase;
        float* __restrict__ yl = ybuf[k & 1];
        float xv[R][W];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if ((lmask >> i) & 1u) {
#pragma unroll
                for (int j = 1; j < W; ++j) xv[i][j] = *reinterpret_cast<const float*>(xl + coff[i][j]);
            } else {
#pragma unroll
                for (int j = 1; j < W; ++j) xv[i][j] = ld_iter<COH>(x, coff[i][j]);
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            // the row's own previous value is yv[i]
            float acc = dlo[i] * yv[i];
            acc = fmaf(cval[i][0], yv[i], acc);
#pragma unroll
            for (int j = 1; j < W; ++j) acc = fmaf(cval[i][j], xv[i][j], acc);
            yv[i] = fs * acc;
            part += (double)yv[i];
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            yl[lrow0 + 64 * i] = yv[i];
            // rows >= n fall outside the range; a single workgroup reads only its LDS copy
            if (G > 1) st_iter<COH>(y, 4u * (uint32_t)row(i), yv[i]);
        }
        accumulate(k);
        bool renorm = false;
        if (m > 0 && --rc == 0) {
            rc = m;
            rpar ^= 1;
            renorm = k < a.Kmax;
        }
        if (G == 1) {
            // one workgroup: the LDS double buffer needs only its own barrier,
            // and its block sum is the whole mass (the same value the grid
            // path's sum over one partial gives)
            if (k == a.Kmax) break;
            if (renorm) {
                const double s = block_sum_f64(part, red);
                if (threadIdx.x == 0) red[kPWaves] = s;
                __syncthreads();
                last_mass = red[kPWaves];
                scale = (last_mass > 0.0 && mass0 > 0.0) ? mass0 / last_mass : 1.0;
            } else {
                __syncthreads();
                scale = 1.0;
            }
            continue;
        }
        double* pm = a.pmass + (size_t)G * (1 + rpar);
        if (renorm) {
            const double s = block_sum_f64(part, red);
            if (threadIdx.x == 0) __hip_atomic_store(pm + g, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (k == a.Kmax) break;
        if (renorm || !a.wait) {
            ++epoch;
            if (!grid_barrier<COH>(a.bar, epoch, g, G, a.flags, a.timeout_ticks)) return;
            if (a.wait && threadIdx.x == 0)  // keep the flags current for later neighbour waits
                __hip_atomic_store(&a.wflag[g * 32], (unsigned)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (!neighbour_sync<COH>(a.wflag, wlo, whi, (unsigned)k, g, a.flags, a.timeout_ticks)) return;
        }
        if (renorm) {
            last_mass = sum_partials(pm, G, red);
            scale = (last_mass > 0.0 && mass0 > 0.0) ? mass0 / last_mass : 1.0;
        } else {
            scale = 1.0;
        }
    }
    if (g == 0 && threadIdx.x == 0) {
        a.mass_out[0] = mass0;
        a.mass_out[1] = last_mass;
    }
}

template <int R, int W, bool CSR, bool COH>
__global__ __launch_bounds__(kPThreads) void k_persistent(PersistArgs a) {
    persistent_body<R, W, CSR, COH, false>(a);
}

// Batched sweep: workgroup g runs items g, g + grid, g + 2 grid, ... of its
// class (ordered longest first by the host, so each round of the grid takes
// the next-longest items).  The assignment is static: a queue counter popped
// by one thread puts a divergent branch in front of the loop's barrier,
// which the compiler may rotate into a nested loop whose other lanes pass
// the barrier without the pop.
template <int R, int W, bool CSR>
__global__ __launch_bounds__(kPThreads) void k_expv_items(const PersistArgs* __restrict__ items, int B) {
    for (int b = blockIdx.x; b < B; b += gridDim.x) persistent_body<R, W, CSR, true, true>(items[b]);
}

// Before the batched sweep: the Poisson weights of every item's windows (the
// single sweep's formula) and each item's flags word cleared.
__global__ __launch_bounds__(256) void k_item_weights(const PersistArgs* __restrict__ items) {
    const PersistArgs& a = items[blockIdx.x];
    if (threadIdx.x == 0) *a.flags = 0u;
    double* wt = const_cast<double*>(a.wtab);
    for (int j = 0; j < a.at.n; ++j) {
        const TimeParam& tp = a.at.tp[j];
        const int cnt = tp.K - tp.L + 1;
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) wt[tp.woff + i] = poisson_weight(tp.W, tp.L + i);
    }
}


// ---------------------------------------------------------------------------
// Two jumps per synchronisation (communication-avoiding form of the same
// sweep).  Workgroup g owns rows [r0, r1) (kP2Rows of them, R = 8 per
// thread as above).  E1 = [e1lo, e1hi) is the hull of the columns its rows
// read, E2 = [e2lo, e2hi) the hull of the columns E1's rows read.  A round
// advances the iterate from x_k to x_{k+2}:
//   A  read x_k on E2 outside the own rows from the global iterate (one
//      coalesced pass; the own rows are already in LDS),
//   B  x_{k+1} on all of E1 from that LDS copy: own rows with the operator
//      in registers, the halo rows E1 \ own with their entries kept in LDS
//      as (byte offset into the E2 copy, value) pairs, copied once from the
//      operator in the same order as the owner's registers, so the owner and
//      the neighbours form bit-identical values; a thread reads all entries
//      of its halo rows, then all their gathers, then does the arithmetic,
//   C  x_{k+2} on the own rows from x_{k+1} in LDS; stored to LDS and to the
//      global iterate, then one synchronisation (neighbour flags, or a grid
//      barrier at a renormalisation point, which must fall on an even jump).
// Every jump's values equal the one-jump kernel's bit for bit: halo rows are
// recomputed from the same inputs with the same operations.  Global
// accesses of the iterate use the device-scope protocol.
constexpr int kP2R = 8;                          // own rows per thread
constexpr int kP2Rows = kPWaves * kP2R * 64;     // own rows of a workgroup
constexpr int kP2Halo = 2048;                    // rows of E1 outside the own rows, at most
constexpr int kP2HR = kP2Halo / kPThreads;       // halo rows per thread
constexpr int kP2X2 = kP2Rows + 2 * kP2Halo;     // rows of E2, at most
constexpr int kP2X1 = kP2Rows + kP2Halo;         // rows of E1, at most
constexpr int kP2Tab = 8;                        // {r0, r1, e1lo, e1hi, e2lo, e2hi, wlo, whi}
constexpr int kP2Slots = 2;                      // open windows held in registers (the one-jump kernel: 4)

template <int W>
constexpr size_t p2_lds_bytes() {
    return sizeof(float) * (kP2X2 + kP2X1) + sizeof(uint2) * (size_t)kP2Halo * W + sizeof(float) * kP2Halo;
}

// Entries of pull row m (column, value) in the order the one-jump kernel
// keeps them in registers (entry 0: the diagonal's hi part, column m) and
// the diagonal's lo part; absent entries read row m with weight 0.
template <int W, bool CSR>
__device__ __forceinline__ void row_entries(const PersistArgs& a, int64_t m, int32_t (&cc)[W], float (&vv)[W],
                                            float& lo) {
    if constexpr (CSR) {
        const int s = (int)(m >> 6), l = (int)(m & 63);
        lo = a.dlo[m];
        int beg = 0, w = 0;
        if (s < a.n_slices) {
            beg = a.slice_off[s];
            w = (a.slice_off[s + 1] - beg) >> 6;
        }
#pragma unroll
        for (int j = 0; j < W; ++j) {
            if (j < w) {
                cc[j] = a.col[beg + j * 64 + l];
                vv[j] = a.val[beg + j * 64 + l];
            } else {
                cc[j] = (int32_t)m;
                vv[j] = 0.f;
            }
        }
    } else {
        stencil_entries<W>(a.cf, m, cc, vv, lo);
    }
}

template <int W, bool CSR, bool FORCE = false>
__global__ __launch_bounds__(kPThreads) void k_persistent2(PersistArgs a) {
    constexpr int R = kP2R;
    extern __shared__ __align__(16) char p2lds[];
    float* X2 = reinterpret_cast<float*>(p2lds);                  // x_k on E2
    float* X1 = X2 + kP2X2;                                       // x_{k+1} on E1
    // halo entries (4 (column - e2lo), value bits), entry j of halo row h at
    // [j][h]: consecutive lanes (consecutive halo rows) read consecutive
    // 8-byte words, free of bank conflicts
    uint2* hent = reinterpret_cast<uint2*>(X1 + kP2X1);
    float* hlo = reinterpret_cast<float*>(hent + (size_t)kP2Halo * W);  // halo rows' diagonal lo parts
    __shared__ double red[kPWaves + 1];
    const int G = a.G;
    const int g = logical_block(G);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = a.n;
    const int32_t* tb = a.p2 + kP2Tab * g;
    const int r0 = tb[0], r1 = tb[1], e1lo = tb[2], e1hi = tb[3], e2lo = tb[4], e2hi = tb[5];
    const int wlo = tb[6], whi = tb[7];
    const int nlo = r0 - e1lo, nh = nlo + (e1hi - r1);        // halo rows of E1: below, in total
    const int nl2 = r0 - e2lo, nt2 = nl2 + (e2hi - r1);       // rows of E2 outside the own rows
    const int32_t row0 = ((g * kPWaves + wave) * R) * 64 + lane;
    auto row = [&](int i) { return row0 + 64 * i; };
    auto live = [&](int i) { return (int64_t)(row0 + 64 * i) < n; };

    // own rows' operator in registers (byte offsets of absolute columns;
    // entry 0 is the diagonal, whose column is the row itself: its value is
    // the thread's own yv[i], so coff[i][0] is never read)
    uint32_t coff[R][W];
    float cval[R][W];
    float dlo[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        int32_t cc[W];
        float vv[W], lo;
        row_entries<W, CSR>(a, live(i) ? (int64_t)row(i) : 0, cc, vv, lo);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            coff[i][j] = live(i) ? 4u * (uint32_t)cc[j] : 4u * (uint32_t)e1lo;
            cval[i][j] = live(i) ? vv[j] : 0.f;
        }
        dlo[i] = live(i) ? lo : 0.f;
    }
    // halo rows' entries in LDS
    for (int h = tid; h < nh; h += kPThreads) {
        const int m = h < nlo ? e1lo + h : r1 + (h - nlo);
        int32_t cc[W];
        float vv[W], lo;
        row_entries<W, CSR>(a, m, cc, vv, lo);
#pragma unroll
        for (int j = 0; j < W; ++j)
            hent[j * kP2Halo + h] = make_uint2(4u * (uint32_t)(cc[j] - e2lo), __builtin_bit_cast(uint32_t, vv[j]));
        hlo[h] = lo;
    }

    // ---- k = 0
    float sacc[kP2Slots][R], cacc[kP2Slots][R];
#pragma unroll
    for (int q = 0; q < kP2Slots; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) { sacc[q][i] = 0.f; cacc[q][i] = 0.f; }
    float yv[R];
    double mloc = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        yv[i] = live(i) ? a.rho0[row(i)] : 0.f;
        if (live(i)) {
            if (!(yv[i] >= 0.f)) atomicOr(a.flags, (yv[i] != yv[i]) ? (unsigned)MJP_FLAG_NAN : (unsigned)MJP_FLAG_NEG);
            else if (isinf(yv[i])) atomicOr(a.flags, (unsigned)MJP_FLAG_NAN);
            X2[row(i) - e2lo] = yv[i];
        }
        mloc += (double)yv[i];
    }
    int jq[kP2Slots], jL[kP2Slots], jK[kP2Slots], jO[kP2Slots];  // as in the one-jump kernel
    int knext = 0;
    float wvec[kP2Slots];
    int wbase = 0;
    auto fetch = [&](int k) {
        if (k >= knext) {
            knext = INT_MAX;
#pragma unroll
            for (int qq = 0; qq < kP2Slots; ++qq) {
                jq[qq] = -1;
                jL[qq] = jK[qq] = jO[qq] = 0;
            }
            for (int j = 0; j < a.at.n; ++j) {
                const TimeParam& tp = a.at.tp[j];
                const int L = tp.L, K = tp.K;
                if (k < L) {
                    knext = min(knext, L);
                    continue;
                }
                if (k > K) continue;
                knext = min(knext, K + 1);
                const int o = tp.out, sj = a.slot[j];
#pragma unroll
                for (int qq = 0; qq < kP2Slots; ++qq)
                    if (qq == sj) { jq[qq] = j; jL[qq] = L; jK[qq] = K; jO[qq] = o; }
            }
        }
        if ((k & 63) == 0) {
            wbase = k;
            const int kk = k + lane;
#pragma unroll
            for (int qq = 0; qq < kP2Slots; ++qq) wvec[qq] = 0.f;
            for (int j = 0; j < a.at.n; ++j) {
                const TimeParam& tp = a.at.tp[j];
                if (kk < tp.L || kk > tp.K) continue;
                const float w = (kk == tp.K) ? (float)tp.lastw : (float)a.wtab[tp.woff + (kk - tp.L)];
#pragma unroll
                for (int qq = 0; qq < kP2Slots; ++qq)
                    if (qq == a.slot[j]) wvec[qq] = w;
            }
        }
    };
    auto accumulate = [&](int k) {
#pragma unroll
        for (int qq = 0; qq < kP2Slots; ++qq) {
            if (jq[qq] < 0) continue;
            const float w = __builtin_bit_cast(
                float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wvec[qq]), k - wbase));
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (k == jL[qq]) {
                    sacc[qq][i] = w * yv[i];
                    cacc[qq][i] = 0.f;
                } else {
                    const float yk = fmaf(w, yv[i], -cacc[qq][i]);
                    const float t = sacc[qq][i] + yk;
                    cacc[qq][i] = (t - sacc[qq][i]) - yk;
                    sacc[qq][i] = t;
                }
                if (k == jK[qq] && live(i)) a.out[(int64_t)jO[qq] * n + row(i)] = sacc[qq][i] - cacc[qq][i];
            }
        }
    };
    fetch(0);
    accumulate(0);
    {
        const double s = block_sum_f64(mloc, red);
        if (tid == 0) __hip_atomic_store(a.pmass + g, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned epoch = 1;
    if (!grid_barrier<true, FORCE>(a.bar, epoch, g, G, a.flags, a.timeout_ticks)) return;
    const double mass0 = sum_partials(a.pmass, G, red);
    double scale = 1.0;
    double last_mass = mass0;
    const int m = a.renorm_every;  // even or 0
    int rc = m, rpar = 0;          // countdown to the next renormalisation, parity of those done
    const __amdgpu_buffer_rsrc_t r_rho0 = iter_rsrc(a.rho0, n), r_buf0 = iter_rsrc(a.buf0, n),
                                 r_buf1 = iter_rsrc(a.buf1, n);
    const char* __restrict__ x2b = reinterpret_cast<const char*>(X2) - 4 * (int64_t)e2lo;
    const char* __restrict__ x1b = reinterpret_cast<const char*>(X1) - 4 * (int64_t)e1lo;
    for (int k = 0; k < a.Kmax; k += 2) {
        const int q = k >> 1;
        const __amdgpu_buffer_rsrc_t src = (q == 0) ? r_rho0 : ((q & 1) ? r_buf0 : r_buf1);
        const __amdgpu_buffer_rsrc_t dst = ((q + 1) & 1) ? r_buf0 : r_buf1;
        // A: x_k on E2 outside the own rows (loads past the vector's end read 0)
        {
            constexpr int kU = kP2X2 / kPThreads - kP2R;  // passes covering E2 \ own
            float t[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = tid + u * kPThreads;
                const int rr = i < nl2 ? e2lo + i : r1 + (i - nl2);
                t[u] = ld_iter<true>(src, 4u * (uint32_t)rr);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = tid + u * kPThreads;
                if (i < nt2) X2[i < nl2 ? i : (r1 - e2lo) + (i - nl2)] = t[u];
            }
        }
        __syncthreads();
        // B: x_{k+1} on E1
        fetch(k + 1);
        {
            const float fs = (float)scale;
            float xv[R][W];
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 1; j < W; ++j) xv[i][j] = *reinterpret_cast<const float*>(x2b + coff[i][j]);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                float acc = dlo[i] * yv[i];  // yv[i]: the row's x_k
                acc = fmaf(cval[i][0], yv[i], acc);
#pragma unroll
                for (int j = 1; j < W; ++j) acc = fmaf(cval[i][j], xv[i][j], acc);
                yv[i] = fs * acc;
            }
            if (nh > 0) {
                constexpr int kB = 2;  // halo rows per batch (registers)
#pragma unroll
                for (int u0 = 0; u0 < kP2HR; u0 += kB) {
                    uint2 e[kB][W];
                    float hx[kB][W];
#pragma unroll
                    for (int u = 0; u < kB; ++u) {
                        const int h = min(tid + (u0 + u) * kPThreads, nh - 1);
#pragma unroll
                        for (int j = 0; j < W; ++j) e[u][j] = hent[j * kP2Halo + h];
                    }
#pragma unroll
                    for (int u = 0; u < kB; ++u)
#pragma unroll
                        for (int j = 0; j < W; ++j)
                            hx[u][j] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(X2) + e[u][j].x);
#pragma unroll
                    for (int u = 0; u < kB; ++u) {
                        const int h = tid + (u0 + u) * kPThreads;
                        float acc = hlo[min(h, nh - 1)] * hx[u][0];  // entry 0: the diagonal
#pragma unroll
                        for (int j = 0; j < W; ++j) acc = fmaf(__builtin_bit_cast(float, e[u][j].y), hx[u][j], acc);
                        if (h < nh) X1[h < nlo ? h : (r1 - e1lo) + (h - nlo)] = fs * acc;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (live(i)) X1[row(i) - e1lo] = yv[i];
        }
        accumulate(k + 1);
        if (k + 1 == a.Kmax) break;
        __syncthreads();
        // C: x_{k+2} on the own rows
        fetch(k + 2);
        double part = 0.0;
        {
            float xv[R][W];
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 1; j < W; ++j) xv[i][j] = *reinterpret_cast<const float*>(x1b + coff[i][j]);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                float acc = dlo[i] * yv[i];  // yv[i]: the row's x_{k+1}
                acc = fmaf(cval[i][0], yv[i], acc);
#pragma unroll
                for (int j = 1; j < W; ++j) acc = fmaf(cval[i][j], xv[i][j], acc);
                yv[i] = 1.0f * acc;
                part += (double)yv[i];
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (live(i)) X2[row(i) - e2lo] = yv[i];
                st_iter<true>(dst, 4u * (uint32_t)row(i), yv[i]);  // rows >= n fall outside the range
            }
        }
        accumulate(k + 2);
        bool renorm = false;
        if (m > 0 && (rc -= 2) == 0) {
            rc = m;
            rpar ^= 1;
            renorm = k + 2 < a.Kmax;
        }
        double* pm = a.pmass + (size_t)G * (1 + rpar);
        if (renorm) {
            const double s = block_sum_f64(part, red);
            if (tid == 0) __hip_atomic_store(pm + g, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (k + 2 == a.Kmax) break;
        if (renorm) {
            ++epoch;
            if (!grid_barrier<true, FORCE>(a.bar, epoch, g, G, a.flags, a.timeout_ticks)) return;
            if (tid == 0) __hip_atomic_store(&a.wflag[g * 32], (unsigned)(k + 2), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last_mass = sum_partials(pm, G, red);
            scale = (last_mass > 0.0 && mass0 > 0.0) ? mass0 / last_mass : 1.0;
        } else {
            if (!neighbour_sync<true, FORCE>(a.wflag, wlo, whi, (unsigned)(k + 2), g, a.flags, a.timeout_ticks)) return;
            scale = 1.0;
        }
    }
    if (g == 0 && tid == 0) {
        a.mass_out[0] = mass0;
        a.mass_out[1] = last_mass;
    }
}

// ---------------------------------------------------------------------------
// S jumps per synchronisation on tiles (the matrix-powers form of the sweep).
// Workgroup g owns up to kMJOwn rows (for a grid operator: a 2-D tile of
// cells; otherwise a block of consecutive rows).  With E_0 the own rows and
// E_{j+1} the columns that the rows of E_j read, a round advances x_k to
// x_{k+S}: the values of x_k on E_S outside the own rows come from the
// exchange buffer, then jump j (1..S) computes x_{k+j} on E_{S-j} from
// x_{k+j-1} on E_{S-j+1}, all in LDS; the own rows of x_{k+S} go to the
// exchange buffer and one synchronisation (neighbour flags, or the grid
// barrier at a renormalisation point, which must end a round) follows.
// Local numbering: own rows first (tile order), then ring 1 = E_1 \ E_0,
// ring 2, ..., ring S, so every E_j is a prefix.  Own rows keep their
// operator in registers, ring rows 1..S-1 as (LDS offset, value) pairs in
// LDS, formed from the same row entries in the same order, so every value
// equals the one-jump kernel's bit for bit.  The exchange buffer holds the
// own rows of workgroup g at [g kMJOwn, g kMJOwn + n_0) (tile order); a
// host-built table gives each ring row's position there.
constexpr int kMJR = 8;                         // own rows per thread
constexpr int kMJOwn = kPWaves * kMJR * 64;     // own rows of a workgroup (4096)
constexpr int kMJHdr = 32;                      // per-workgroup header words
constexpr int kMJNb = 16;                       // neighbours a workgroup waits for, at most
// header: [0..S] n_0 .. n_S, [9] neighbour count, [10] own block (gid, lcol),
// [11] ring block (gid, lcol), [12] positions, [16..31] neighbours
enum { kMJHCount = 9, kMJHOwn = 10, kMJHRing = 11, kMJHPos = 12, kMJHNb = 16 };
// rows of rings 1..S-1 and of rings 1..S a workgroup holds, at most (63 x 63
// tiles: 792 / 1072 for S = 4, 1960 / 2272 for S = 8)
constexpr int mj_halo_cap(int S) { return S == 4 ? 1024 : 2048; }
constexpr int mj_load_cap(int S) { return S == 4 ? 1536 : 2304; }
constexpr int mj_x_cap(int S) { return kMJOwn + mj_load_cap(S); }

template <int W, int S>
constexpr size_t mj_lds_bytes() {
    return sizeof(float) * 2 * mj_x_cap(S) + sizeof(uint2) * (size_t)mj_halo_cap(S) * W +
           sizeof(float) * mj_halo_cap(S) + (sizeof(int32_t) + sizeof(uint16_t)) * mj_load_cap(S);
}
// the exchange probe's LDS: E_S's values and the load lists
constexpr size_t mj_probe_lds_bytes(int S) {
    return sizeof(float) * (size_t)mj_x_cap(S) + (sizeof(int32_t) + sizeof(uint16_t)) * (size_t)mj_load_cap(S);
}

template <int W, bool CSR, int S>
__global__ __launch_bounds__(kPThreads) void k_persistent_mj(PersistArgs a) {
    constexpr int R = kMJR;
    constexpr int kMJHalo = mj_halo_cap(S), kMJLoad = mj_load_cap(S), kMJX = mj_x_cap(S);
    extern __shared__ __align__(16) char mjlds[];
    float* X0 = reinterpret_cast<float*>(mjlds);            // x_{k+j} for even j (E_S at j = 0)
    float* X1 = X0 + kMJX;                                   // x_{k+j} for odd j
    uint2* hent = reinterpret_cast<uint2*>(X1 + kMJX);      // ring rows' entries, entry j of row h at [j][h]
    float* hlo = reinterpret_cast<float*>(hent + (size_t)kMJHalo * W);
    // rings 1..S in exchange-buffer order (coalesced loads): position, and
    // the row's place after the own rows
    int32_t* lpos = reinterpret_cast<int32_t*>(hlo + kMJHalo);
    uint16_t* lloc = reinterpret_cast<uint16_t*>(lpos + kMJLoad);
    __shared__ double red[kPWaves + 1];
    const int G = a.G;
    const int g = logical_block(G);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = a.n;
    const int32_t* hd = a.p2 + (size_t)kMJHdr * g;
    int nS[S + 1];
#pragma unroll
    for (int j = 0; j <= S; ++j) nS[j] = hd[j];
    const int n0 = nS[0], nh = nS[S - 1] - n0, nl = nS[S] - n0;
    const int nn = hd[kMJHCount];
    const int32_t* own_gid = a.p2 + hd[kMJHOwn];
    const int32_t* own_lcol = own_gid + n0;
    const int32_t* ring_gid = a.p2 + hd[kMJHRing];
    const int32_t* ring_lcol = ring_gid + nh;
    const int32_t* pos = a.p2 + hd[kMJHPos];
    auto li = [&](int i) { return (wave * R + i) * 64 + lane; };
    auto live = [&](int i) { return li(i) < n0; };

    uint32_t coff[R][W];
    float cval[R][W];
    float dlo[R];
    int32_t gid[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        gid[i] = live(i) ? own_gid[li(i)] : 0;
        int32_t cc[W];
        float vv[W], lo;
        row_entries<W, CSR>(a, (int64_t)gid[i], cc, vv, lo);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            coff[i][j] = live(i) ? 4u * (uint32_t)own_lcol[(size_t)li(i) * W + j] : 0u;
            cval[i][j] = live(i) ? vv[j] : 0.f;
        }
        dlo[i] = live(i) ? lo : 0.f;
    }
    for (int h = tid; h < nh; h += kPThreads) {
        int32_t cc[W];
        float vv[W], lo;
        row_entries<W, CSR>(a, (int64_t)ring_gid[h], cc, vv, lo);
#pragma unroll
        for (int j = 0; j < W; ++j)
            hent[j * kMJHalo + h] = make_uint2(4u * (uint32_t)ring_lcol[(size_t)h * W + j], __builtin_bit_cast(uint32_t, vv[j]));
        hlo[h] = lo;
    }
    for (int h = tid; h < kMJLoad; h += kPThreads) {
        lpos[h] = h < nl ? pos[h] : 0;
        lloc[h] = h < nl ? (uint16_t)pos[nl + h] : (uint16_t)0;
    }

    // ---- k = 0: own rows of x_0 into LDS and into the exchange buffer the
    // first round reads (buf1), then the initial mass
    float sacc[kP2Slots][R], cacc[kP2Slots][R];
#pragma unroll
    for (int q = 0; q < kP2Slots; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) { sacc[q][i] = 0.f; cacc[q][i] = 0.f; }
    float yv[R];
    double mloc = 0.0;
    const __amdgpu_buffer_rsrc_t r_buf0 = iter_rsrc(a.buf0, (int64_t)G * kMJOwn),
                                 r_buf1 = iter_rsrc(a.buf1, (int64_t)G * kMJOwn);
    const uint32_t pbase = 4u * (uint32_t)(g * kMJOwn);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        yv[i] = live(i) ? a.rho0[gid[i]] : 0.f;
        if (live(i)) {
            if (!(yv[i] >= 0.f)) atomicOr(a.flags, (yv[i] != yv[i]) ? (unsigned)MJP_FLAG_NAN : (unsigned)MJP_FLAG_NEG);
            else if (isinf(yv[i])) atomicOr(a.flags, (unsigned)MJP_FLAG_NAN);
            X0[li(i)] = yv[i];
            st_iter<true>(r_buf1, pbase + 4u * (uint32_t)li(i), yv[i]);
        }
        mloc += (double)yv[i];
    }
    int jq[kP2Slots], jL[kP2Slots], jK[kP2Slots], jO[kP2Slots];  // as in the one-jump kernel
    int knext = 0;
    float wvec[kP2Slots];
    int wbase = 0;
    auto fetch = [&](int k) {
        if (k >= knext) {
            knext = INT_MAX;
#pragma unroll
            for (int qq = 0; qq < kP2Slots; ++qq) {
                jq[qq] = -1;
                jL[qq] = jK[qq] = jO[qq] = 0;
            }
            for (int j = 0; j < a.at.n; ++j) {
                const TimeParam& tp = a.at.tp[j];
                const int L = tp.L, K = tp.K;
                if (k < L) {
                    knext = min(knext, L);
                    continue;
                }
                if (k > K) continue;
                knext = min(knext, K + 1);
                const int o = tp.out, sj = a.slot[j];
#pragma unroll
                for (int qq = 0; qq < kP2Slots; ++qq)
                    if (qq == sj) { jq[qq] = j; jL[qq] = L; jK[qq] = K; jO[qq] = o; }
            }
        }
        if ((k & 63) == 0) {
            wbase = k;
            const int kk = k + lane;
#pragma unroll
            for (int qq = 0; qq < kP2Slots; ++qq) wvec[qq] = 0.f;
            for (int j = 0; j < a.at.n; ++j) {
                const TimeParam& tp = a.at.tp[j];
                if (kk < tp.L || kk > tp.K) continue;
                const float w = (kk == tp.K) ? (float)tp.lastw : (float)a.wtab[tp.woff + (kk - tp.L)];
#pragma unroll
                for (int qq = 0; qq < kP2Slots; ++qq)
                    if (qq == a.slot[j]) wvec[qq] = w;
            }
        }
    };
    auto accumulate = [&](int k) {
#pragma unroll
        for (int qq = 0; qq < kP2Slots; ++qq) {
            if (jq[qq] < 0) continue;
            const float w = __builtin_bit_cast(
                float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wvec[qq]), k - wbase));
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (k == jL[qq]) {
                    sacc[qq][i] = w * yv[i];
                    cacc[qq][i] = 0.f;
                } else {
                    const float yk = fmaf(w, yv[i], -cacc[qq][i]);
                    const float t = sacc[qq][i] + yk;
                    cacc[qq][i] = (t - sacc[qq][i]) - yk;
                    sacc[qq][i] = t;
                }
                if (k == jK[qq] && live(i)) a.out[(int64_t)jO[qq] * n + gid[i]] = sacc[qq][i] - cacc[qq][i];
            }
        }
    };
    fetch(0);
    accumulate(0);
    {
        const double s = block_sum_f64(mloc, red);
        if (tid == 0) __hip_atomic_store(a.pmass + g, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned epoch = 1;
    if (!grid_barrier<true>(a.bar, epoch, g, G, a.flags, a.timeout_ticks)) return;
    const double mass0 = sum_partials(a.pmass, G, red);
    double scale = 1.0;
    double last_mass = mass0;
    const int m = a.renorm_every;  // a multiple of S, or 0
    int rc = m, rpar = 0;
    for (int k = 0; k < a.Kmax; k += S) {
        const int q = k / S;
        const __amdgpu_buffer_rsrc_t src = (q & 1) ? r_buf0 : r_buf1;
        const __amdgpu_buffer_rsrc_t dst = (q & 1) ? r_buf1 : r_buf0;
        // x_k on rings 1..S from the exchange buffer
        {
            constexpr int kU = (kMJLoad + kPThreads - 1) / kPThreads;  // passes covering every ring row
            float t[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int h = tid + u * kPThreads;
                t[u] = ld_iter<true>(src, 4u * (uint32_t)lpos[min(h, kMJLoad - 1)]);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int h = tid + u * kPThreads;
                if (h < nl) X0[n0 + lloc[h]] = t[u];
            }
        }
        __syncthreads();
        double part = 0.0;
#pragma unroll
        for (int jj = 1; jj <= S; ++jj) {
            const float* Xr = (jj & 1) ? X0 : X1;
            float* Xw = (jj & 1) ? X1 : X0;
            const char* __restrict__ xrb = reinterpret_cast<const char*>(Xr);
            const float fs = jj == 1 ? (float)scale : 1.0f;
            fetch(k + jj);
            {
                float xv[R][W];
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 1; j < W; ++j) xv[i][j] = *reinterpret_cast<const float*>(xrb + coff[i][j]);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    float acc = dlo[i] * yv[i];
                    acc = fmaf(cval[i][0], yv[i], acc);
#pragma unroll
                    for (int j = 1; j < W; ++j) acc = fmaf(cval[i][j], xv[i][j], acc);
                    yv[i] = fs * acc;
                }
            }
            const int nring = nS[S - jj] - n0;  // ring rows this jump computes
            if (nring > 0) {
                constexpr int kB = 2;
                for (int u0 = 0; u0 * kPThreads < nring; u0 += kB) {
                    uint2 e[kB][W];
                    float hx[kB][W];
#pragma unroll
                    for (int u = 0; u < kB; ++u) {
                        const int h = min(tid + (u0 + u) * kPThreads, nring - 1);
#pragma unroll
                        for (int j = 0; j < W; ++j) e[u][j] = hent[j * kMJHalo + h];
                    }
#pragma unroll
                    for (int u = 0; u < kB; ++u)
#pragma unroll
                        for (int j = 0; j < W; ++j) hx[u][j] = *reinterpret_cast<const float*>(xrb + e[u][j].x);
#pragma unroll
                    for (int u = 0; u < kB; ++u) {
                        const int h = tid + (u0 + u) * kPThreads;
                        float acc = hlo[min(h, nring - 1)] * hx[u][0];
#pragma unroll
                        for (int j = 0; j < W; ++j) acc = fmaf(__builtin_bit_cast(float, e[u][j].y), hx[u][j], acc);
                        if (h < nring) Xw[n0 + h] = fs * acc;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (live(i)) Xw[li(i)] = yv[i];
            accumulate(k + jj);
            if (k + jj == a.Kmax) break;
            if (jj < S) __syncthreads();
        }
        if (k + S >= a.Kmax) break;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            part += (double)yv[i];
            if (live(i)) st_iter<true>(dst, pbase + 4u * (uint32_t)li(i), yv[i]);
        }
        bool renorm = false;
        if (m > 0 && (rc -= S) == 0) {
            rc = m;
            rpar ^= 1;
            renorm = true;
        }
        double* pm = a.pmass + (size_t)G * (1 + rpar);
        if (renorm) {
            const double s = block_sum_f64(part, red);
            if (tid == 0) __hip_atomic_store(pm + g, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ++epoch;
            if (!grid_barrier<true>(a.bar, epoch, g, G, a.flags, a.timeout_ticks)) return;
            if (tid == 0) __hip_atomic_store(&a.wflag[g * 32], (unsigned)(k + S), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last_mass = sum_partials(pm, G, red);
            scale = (last_mass > 0.0 && mass0 > 0.0) ? mass0 / last_mass : 1.0;
        } else {
            if (!neighbour_sync_set(a.wflag, hd + kMJHNb, nn, (unsigned)(k + S), g, a.flags, a.timeout_ticks)) return;
            scale = 1.0;
        }
    }
    if (g == 0 && tid == 0) {
        a.mass_out[0] = mass0;
        a.mass_out[1] = last_mass;
    }
}

// Exchange floor of the tiled sweep (a measurement aid): `rounds` rounds of
// exactly its per-round communication with no arithmetic -- the ring loads
// from the exchange buffer into LDS, a workgroup barrier, the own rows'
// stores, the neighbour synchronisation -- on the same table and launch.
template <int S>
__global__ __launch_bounds__(kPThreads) void k_exchange_probe_mj(PersistArgs a, int rounds) {
    constexpr int R = kMJR;
    constexpr int kMJLoad = mj_load_cap(S), kMJX = mj_x_cap(S);
    extern __shared__ __align__(16) char mjlds[];
    float* X0 = reinterpret_cast<float*>(mjlds);
    int32_t* lpos = reinterpret_cast<int32_t*>(X0 + kMJX);
    uint16_t* lloc = reinterpret_cast<uint16_t*>(lpos + kMJLoad);
    const int G = a.G;
    const int g = logical_block(G);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t* hd = a.p2 + (size_t)kMJHdr * g;
    const int n0 = hd[0], nl = hd[S] - n0;
    const int nn = hd[kMJHCount];
    const int32_t* pos = a.p2 + hd[kMJHPos];
    for (int h = tid; h < kMJLoad; h += kPThreads) {
        lpos[h] = h < nl ? pos[h] : 0;
        lloc[h] = h < nl ? (uint16_t)pos[nl + h] : (uint16_t)0;
    }
    for (int i = tid; i < kMJX; i += kPThreads) X0[i] = 0.f;
    __syncthreads();
    const __amdgpu_buffer_rsrc_t r_buf0 = iter_rsrc(a.buf0, (int64_t)G * kMJOwn),
                                 r_buf1 = iter_rsrc(a.buf1, (int64_t)G * kMJOwn);
    const uint32_t pbase = 4u * (uint32_t)(g * kMJOwn);
    for (int q = 0; q < rounds; ++q) {
        const __amdgpu_buffer_rsrc_t src = (q & 1) ? r_buf0 : r_buf1;
        const __amdgpu_buffer_rsrc_t dst = (q & 1) ? r_buf1 : r_buf0;
        constexpr int kU = (kMJLoad + kPThreads - 1) / kPThreads;
        float t[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) t[u] = ld_iter<true>(src, 4u * (uint32_t)lpos[min(tid + u * kPThreads, kMJLoad - 1)]);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int h = tid + u * kPThreads;
            if (h < nl) X0[n0 + lloc[h]] = t[u];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int li = (wave * R + i) * 64 + lane;
            if (li < n0) st_iter<true>(dst, pbase + 4u * (uint32_t)li, X0[li]);
        }
        if (!neighbour_sync_set(a.wflag, hd + kMJHNb, nn, (unsigned)((q + 1) * S), g, a.flags, a.timeout_ticks)) return;
    }
}

// Exchange floor of the two-jump sweep (a measurement aid, not part of the
// method): `rounds` rounds of exactly its per-round communication with no
// arithmetic.  Each round: load the iterate on E2 outside the own rows from
// global memory into LDS (device scope, the same coalesced pass as phase A),
// a workgroup barrier, store the own rows from LDS (device scope, as phase C
// does), then the same neighbour synchronisation (drain, flag, wait for the
// neighbour interval).  The iterate is copied unchanged between the two
// buffers, so every load reads what a neighbour stored the round before.
template <bool FORCE = false>
__global__ __launch_bounds__(kPThreads) void k_exchange_probe(PersistArgs a, int rounds) {
    extern __shared__ __align__(16) char p2lds[];
    float* X2 = reinterpret_cast<float*>(p2lds);
    const int G = a.G;
    const int g = logical_block(G);
    const int tid = threadIdx.x;
    const int64_t n = a.n;
    const int32_t* tb = a.p2 + kP2Tab * g;
    const int r0 = tb[0], r1 = tb[1], e2lo = tb[4], e2hi = tb[5];
    const int wlo = tb[6], whi = tb[7];
    const int nl2 = r0 - e2lo, nt2 = nl2 + (e2hi - r1);
    for (int r = r0 + tid; r < r1; r += kPThreads) X2[r - e2lo] = a.rho0[r];
    const __amdgpu_buffer_rsrc_t r_buf0 = iter_rsrc(a.buf0, n), r_buf1 = iter_rsrc(a.buf1, n);
    __syncthreads();
    {  // round 0 stores the own rows so the first loads read defined values
        for (int r = r0 + tid; r < r1; r += kPThreads) st_iter<true>(r_buf0, 4u * (uint32_t)r, X2[r - e2lo]);
        if (!neighbour_sync<true, FORCE>(a.wflag, wlo, whi, 1u, g, a.flags, a.timeout_ticks)) return;
    }
    for (int q = 1; q <= rounds; ++q) {
        const __amdgpu_buffer_rsrc_t src = (q & 1) ? r_buf0 : r_buf1;
        const __amdgpu_buffer_rsrc_t dst = (q & 1) ? r_buf1 : r_buf0;
        {
            constexpr int kU = kP2X2 / kPThreads - kP2R;
            float t[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = tid + u * kPThreads;
                const int rr = i < nl2 ? e2lo + i : r1 + (i - nl2);
                t[u] = ld_iter<true>(src, 4u * (uint32_t)rr);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = tid + u * kPThreads;
                if (i < nt2) X2[i < nl2 ? i : (r1 - e2lo) + (i - nl2)] = t[u];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kP2R; ++i) {
            const int r = r0 + tid + i * kPThreads;
            st_iter<true>(dst, 4u * (uint32_t)r, r < r1 ? X2[r - e2lo] : 0.f);  // rows >= n fall outside the range
        }
        if (!neighbour_sync<true, FORCE>(a.wflag, wlo, whi, (unsigned)(q + 1), g, a.flags, a.timeout_ticks)) return;
    }
}

using PersistFn = void (*)(PersistArgs);

template <bool CSR, bool COH>
static PersistFn pick(int R, int W) {
#define MJP_CASE(r, w) if (R == r && W == w) return k_persistent<r, w, CSR, COH>;
    if constexpr (CSR) {
        MJP_CASE(1, 3) MJP_CASE(2, 3) MJP_CASE(4, 3) MJP_CASE(8, 3)
        MJP_CASE(1, 5) MJP_CASE(2, 5) MJP_CASE(4, 5) MJP_CASE(8, 5)
        MJP_CASE(1, 8) MJP_CASE(2, 8) MJP_CASE(4, 8)
        MJP_CASE(1, 12) MJP_CASE(2, 12) MJP_CASE(4, 12)
        MJP_CASE(1, 16) MJP_CASE(2, 16)
    } else {
        MJP_CASE(1, 5) MJP_CASE(2, 5) MJP_CASE(4, 5) MJP_CASE(8, 5)
        MJP_CASE(1, 8) MJP_CASE(2, 8) MJP_CASE(4, 8)
    }
#undef MJP_CASE
    return nullptr;
}

using ItemFn = void (*)(const PersistArgs*, int);

// the item kernel for (R, W): the same shapes as the one-jump kernel
template <bool CSR>
static ItemFn pick_items(int R, int W) {
#define MJP_CASE(r, w) if (R == r && W == w) return k_expv_items<r, w, CSR>;
    if constexpr (CSR) {
        MJP_CASE(1, 3) MJP_CASE(2, 3) MJP_CASE(4, 3) MJP_CASE(8, 3)
        MJP_CASE(1, 5) MJP_CASE(2, 5) MJP_CASE(4, 5) MJP_CASE(8, 5)
        MJP_CASE(1, 8) MJP_CASE(2, 8) MJP_CASE(4, 8)
        MJP_CASE(1, 12) MJP_CASE(2, 12) MJP_CASE(4, 12)
        MJP_CASE(1, 16) MJP_CASE(2, 16)
    } else {
        MJP_CASE(1, 5) MJP_CASE(2, 5) MJP_CASE(4, 5) MJP_CASE(8, 5)
        MJP_CASE(1, 8) MJP_CASE(2, 8) MJP_CASE(4, 8)
    }
#undef MJP_CASE
    return nullptr;
}

// Entries per row of the one-jump kernel for this plan (0: too wide).
static int sweep_width(const mjp_plan* p) {
    if (p->kind != PLAN_CSR) return stencil_width(p->coef.model) <= 5 ? 5 : 8;
    if (p->max_width <= 3) return 3;
    if (p->max_width <= 5) return 5;
    if (p->max_width <= 8) return 8;
    if (p->max_width <= 12) return 12;
    if (p->max_width <= 16) return 16;
    return 0;
}

__global__ void k_zero_u32(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Decide whether the persistent kernel can run this sweep; fills cfg.
bool persistent_fits(const mjp_plan* p, int max_open, bool coh, PersistCfg& cfg) {
    if (max_open > kPSlots) return false;
    if (p->n >= ((int64_t)1 << 30)) return false;  // byte offsets of the iterate must fit 32 bits
    const int W = sweep_width(p);
    if (W == 0) return false;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    const int64_t slices = (p->n + 63) / 64;
    auto fn_for = [&](int R) {
        return p->kind == PLAN_CSR ? (coh ? pick<true, true>(R, W) : pick<true, false>(R, W))
                                   : (coh ? pick<false, true>(R, W) : pick<false, false>(R, W));
    };
    // a vector that one workgroup can hold runs in a single workgroup: every
    // gather is local (LDS) and a jump costs two workgroup barriers
    for (int R : {1, 2, 4, 8}) {
        PersistFn f = fn_for(R);
        if (!f || slices > (int64_t)kPWaves * R) continue;
        cfg.R = R;
        cfg.W = W;
        cfg.G = 1;
        cfg.coh = coh;
        cfg.fn = reinterpret_cast<const void*>(f);
        return true;
    }
    for (int R : {1, 2, 4, 8}) {
        PersistFn f = fn_for(R);
        if (!f) continue;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f), kPThreads, 0) !=
                hipSuccess || per_cu < 1)
            continue;
        const int64_t need = (slices + (int64_t)kPWaves * R - 1) / ((int64_t)kPWaves * R);
        int64_t G = (need + 7) / 8 * 8;
        if (G > (int64_t)ncu * per_cu) continue;  // does not fit co-resident: try more rows per thread
        cfg.R = R;
        cfg.W = W;
        cfg.G = (int)G;
        cfg.coh = coh;
        cfg.fn = reinterpret_cast<const void*>(f);
        return true;
    }
    return false;
}

// ---- the batched sweep
bool item_fits(const mjp_plan* p, int max_open, int& R, int& W) {
    if (max_open > kPSlots || p->n >= ((int64_t)1 << 30)) return false;
    W = sweep_width(p);
    if (W == 0) return false;
    const int64_t slices = (p->n + 63) / 64;
    for (int r : {1, 2, 4, 8}) {
        const ItemFn f = p->kind == PLAN_CSR ? pick_items<true>(r, W) : pick_items<false>(r, W);
        if (f && slices <= (int64_t)kPWaves * r) {
            R = r;
            return true;
        }
    }
    return false;
}

void ItemWork::release() {
    args.release();
    wtab.release();
    info.release();
    if (staged) (void)hipEventDestroy(staged);
    if (stage) (void)hipHostFree(stage);
    staged = nullptr;
    stage = nullptr;
    stage_bytes = 0;
}

mjp_status launch_items(const std::vector<ItemSweep>& items, bool out_mass, ItemWork& ws, hipStream_t st,
                        std::vector<int64_t>& info_off) {
    const int B = (int)items.size();
    info_off.assign(B, 0);
    if (B == 0) return MJP_OK;
    // classes by (kind, R, W); longest first inside a class
    auto cls_key = [&](int i) {
        const ItemSweep& it = items[(size_t)i];
        return (it.p->kind == PLAN_CSR ? 0 : 1000) + it.R * 32 + it.W;
    };
    std::vector<double> work((size_t)B);  // n K_max: the item's cell updates
    for (int i = 0; i < B; ++i) {
        const ItemSweep& it = items[(size_t)i];
        int32_t k = 0;
        for (int j = 0; j < it.at.n; ++j) k = std::max(k, it.at.tp[j].K);
        work[(size_t)i] = (double)it.p->n * (double)k;
    }
    std::vector<int> order((size_t)B);
    for (int i = 0; i < B; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const int kx = cls_key(x), ky = cls_key(y);
        return kx != ky ? kx < ky : work[(size_t)x] > work[(size_t)y];
    });
    std::vector<int64_t> woff((size_t)B);
    int64_t wt = 0, inf = 0;
    for (int i : order) {
        woff[(size_t)i] = wt;
        wt += (std::max<int64_t>(items[(size_t)i].wtotal, 1) + 31) / 32 * 32;  // 256-byte aligned regions
        info_off[(size_t)i] = inf;
        inf += (6 + items[(size_t)i].at.n + 7) / 8 * 8;
    }
    const size_t abytes = sizeof(PersistArgs) * (size_t)B;
    mjp_status s;
    if ((s = ws.args.reserve(abytes)) || (s = ws.wtab.reserve(sizeof(double) * (size_t)wt)) ||
        (s = ws.info.reserve(sizeof(double) * (size_t)inf)))
        return s;
    if (!ws.staged) MJP_HIP(hipEventCreateWithFlags(&ws.staged, hipEventDisableTiming));
    else MJP_HIP(hipEventSynchronize(ws.staged));  // the last upload from the stage has completed
    if (ws.stage_bytes < abytes) {
        if (ws.stage) MJP_HIP(hipHostFree(ws.stage));
        ws.stage = nullptr;
        ws.stage_bytes = 0;
        MJP_HIP(hipHostMalloc(&ws.stage, abytes, hipHostMallocDefault));
        ws.stage_bytes = abytes;
    }
    PersistArgs* A = static_cast<PersistArgs*>(ws.stage);
    double* info = ws.info.as<double>();
    struct Cls { int key, beg, cnt; const ItemSweep* first; };
    std::vector<Cls> cls;
    for (int pos = 0; pos < B; ++pos) {
        const int i = order[(size_t)pos];
        const ItemSweep& it = items[(size_t)i];
        const mjp_plan* p = it.p;
        // every field the single-workgroup sweep reads is written; of the
        // time table only the item's own entries (the struct is 2 KB)
        PersistArgs& a = A[pos];
        a.slice_off = p->slice_off.as<int32_t>();
        a.col = p->col.as<int32_t>();
        a.val = p->val.as<float>();
        a.dlo = p->dlo.as<float>();
        a.cf = p->coef;
        a.rho0 = it.rho0;
        a.out = it.out;
        a.wtab = ws.wtab.as<double>() + woff[(size_t)i];
        double* rep = info + info_off[(size_t)i];
        a.flags = reinterpret_cast<unsigned*>(rep);
        a.mass_out = rep + 1;
        a.pmass = rep + 3;
        a.out_mass = out_mass ? rep + 6 : nullptr;
        a.n = p->n;
        a.n_slices = (int32_t)((p->n + 63) / 64);
        a.Kmax = 0;
        for (int j = 0; j < it.at.n; ++j) a.Kmax = std::max(a.Kmax, it.at.tp[j].K);
        a.renorm_every = p->opts.renorm_every;
        a.G = 1;
        a.buf0 = a.buf1 = nullptr;
        a.bar = a.wflag = nullptr;
        a.wait = a.p2 = nullptr;
        a.sflag = nullptr;
        a.timeout_ticks = 0;
        a.at.n = it.at.n;
        std::memcpy(a.at.tp, it.at.tp, sizeof(TimeParam) * (size_t)it.at.n);
        std::memcpy(a.slot, it.slot, sizeof(int32_t) * (size_t)it.at.n);
        const int key = cls_key(i);
        if (cls.empty() || cls.back().key != key) cls.push_back(Cls{key, pos, 0, &it});
        cls.back().cnt++;
    }
    MJP_HIP(hipMemcpyAsync(ws.args.ptr, ws.stage, abytes, hipMemcpyHostToDevice, st));
    MJP_HIP(hipEventRecord(ws.staged, st));
    const PersistArgs* args_d = ws.args.as<PersistArgs>();
    hipLaunchKernelGGL(k_item_weights, dim3((unsigned)B), dim3(256), 0, st, args_d);
    int dev = 0, ncu = 0;
    MJP_HIP(hipGetDevice(&dev));
    MJP_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    for (size_t c = 0; c < cls.size(); ++c) {
        const ItemSweep& it = *cls[c].first;
        const ItemFn f = it.p->kind == PLAN_CSR ? pick_items<true>(it.R, it.W) : pick_items<false>(it.R, it.W);
        MJP_CHECK(f, MJP_E_UNSUPPORTED, "no item kernel for R=%d W=%d", it.R, it.W);
        int per_cu = 0;
        MJP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f), kPThreads, 0));
        const int grid = std::max(1, std::min(cls[c].cnt, ncu * std::max(per_cu, 1)));
        const PersistArgs* first = args_d + cls[c].beg;
        int cnt = cls[c].cnt;
        void* kargs[] = {&first, &cnt};
        MJP_HIP(hipLaunchKernel(reinterpret_cast<const void*>(f), dim3((unsigned)grid), dim3(kPThreads), kargs, 0, st));
    }
    MJP_HIP(hipGetLastError());
    return MJP_OK;
}

// ---- the two-jump kernel: table and fit
template <bool CSR>
static PersistFn pick2(int W, bool force) {
    if constexpr (CSR) {
        if (W == 3) return force ? k_persistent2<3, true, true> : k_persistent2<3, true>;
        if (W == 5) return force ? k_persistent2<5, true, true> : k_persistent2<5, true>;
    } else {
        if (W == 5) return force ? k_persistent2<5, false, true> : k_persistent2<5, false>;
    }
    return nullptr;
}

static size_t p2_lds_for(int W) { return W == 3 ? p2_lds_bytes<3>() : p2_lds_bytes<5>(); }

// Per workgroup {r0, r1, e1lo, e1hi, e2lo, e2hi, wlo, whi} from the slices'
// column hulls (conservative); false if some region exceeds the LDS
// buffers or a neighbour interval spans more than 64 workgroups.
static bool build_p2_table(const mjp_plan* p, int G, std::vector<int32_t>& tab) {
    const int64_t n = p->n;
    auto hull = [&](int64_t sl, int64_t& lo, int64_t& hi) {
        if (p->kind == PLAN_CSR) {
            lo = p->slice_cmin[(size_t)sl];
            hi = p->slice_cmax[(size_t)sl];
        } else {
            const int64_t reach = stencil_reach(p->coef);
            lo = std::max<int64_t>(0, sl * 64 - reach);
            hi = std::min<int64_t>(n - 1, sl * 64 + 63 + reach);
        }
    };
    // hull of the columns read by rows [a, b)
    auto cols = [&](int64_t a, int64_t b, int64_t& lo, int64_t& hi) {
        lo = a;
        hi = b - 1;
        for (int64_t sl = a / 64; sl <= (b - 1) / 64; ++sl) {
            int64_t l, h;
            hull(sl, l, h);
            lo = std::min(lo, l);
            hi = std::max(hi, h);
        }
    };
    tab.assign((size_t)kP2Tab * G, 0);
    std::vector<int32_t> lo(G), hi(G);
    for (int g = 0; g < G; ++g) {
        int32_t* t = tab.data() + (size_t)kP2Tab * g;
        const int64_t r0 = std::min<int64_t>(n, (int64_t)g * kP2Rows), r1 = std::min<int64_t>(n, r0 + kP2Rows);
        t[0] = (int32_t)r0;
        t[1] = (int32_t)r1;
        lo[g] = hi[g] = g;
        if (r0 >= r1) {
            for (int c = 2; c < 6; ++c) t[c] = (int32_t)r0;
            continue;
        }
        int64_t e1lo, e1hi, e2lo, e2hi;
        cols(r0, r1, e1lo, e1hi);
        cols(e1lo, e1hi + 1, e2lo, e2hi);
        e1hi += 1;
        e2hi += 1;
        if ((r0 - e1lo) + (e1hi - r1) > kP2Halo) return false;
        if ((r0 - e2lo) + (e2hi - r1) > 2 * kP2Halo) return false;
        t[2] = (int32_t)e1lo;
        t[3] = (int32_t)e1hi;
        t[4] = (int32_t)e2lo;
        t[5] = (int32_t)e2hi;
        lo[g] = (int32_t)(e2lo / kP2Rows);
        hi[g] = (int32_t)((e2hi - 1) / kP2Rows);
    }
    // wait for the owners of my E2 and for the workgroups whose E2 holds my rows
    std::vector<int32_t> wlo(lo), whi(hi);
    for (int g = 0; g < G; ++g)
        for (int h = lo[g]; h <= hi[g]; ++h) {
            wlo[h] = std::min(wlo[h], g);
            whi[h] = std::max(whi[h], g);
        }
    for (int g = 0; g < G; ++g) {
        if (whi[g] - wlo[g] + 1 > 64) return false;
        tab[(size_t)kP2Tab * g + 6] = wlo[g];
        tab[(size_t)kP2Tab * g + 7] = whi[g];
    }
    return true;
}

// ---- the tiled multi-jump kernel: tables and fit
static PersistFn pick_mj(int W, bool csr, int S) {
    if (S == 8) {
        if (csr) {
            if (W == 3) return k_persistent_mj<3, true, 8>;
            if (W == 5) return k_persistent_mj<5, true, 8>;
        } else if (W == 5) {
            return k_persistent_mj<5, false, 8>;
        }
    } else if (S == 4) {
        if (csr) {
            if (W == 3) return k_persistent_mj<3, true, 4>;
            if (W == 5) return k_persistent_mj<5, true, 4>;
        } else if (W == 5) {
            return k_persistent_mj<5, false, 4>;
        }
    }
    return nullptr;
}
static size_t mj_lds_for(int W, int S) {
    if (S == 8) return W == 3 ? mj_lds_bytes<3, 8>() : mj_lds_bytes<5, 8>();
    return W == 3 ? mj_lds_bytes<3, 4>() : mj_lds_bytes<5, 4>();
}

// Columns of row m in the order the kernels hold its entries (entry 0 the
// row itself; absent entries the row itself).
struct HostRows {
    const mjp_plan* p;
    std::vector<int32_t> off, col;  // CSR plans: the sliced ELL's offsets and columns
    int W;
    void cols(int64_t m, int32_t* out) const {
        if (p->kind == PLAN_CSR) {
            const int64_t s = m >> 6, l = m & 63;
            const int beg = off[(size_t)s], w = (off[(size_t)s + 1] - beg) >> 6;
            for (int j = 0; j < W; ++j) out[j] = j < w ? col[(size_t)beg + 64 * (size_t)j + (size_t)l] : (int32_t)m;
        } else {
            int32_t cc[kStencilMaxW];
            float vv[kStencilMaxW], lo;
            stencil_entries<kStencilMaxW>(p->coef, m, cc, vv, lo);
            for (int j = 0; j < W; ++j) out[j] = j < kStencilMaxW ? cc[j] : (int32_t)m;
        }
    }
};

// Builds the table for tiles of at most kMJOwn rows and at most `cap`
// workgroups; false if the operator has no grid structure, or a ring or
// neighbour interval exceeds the kernel's buffers.
static bool build_mj_table(mjp_plan* p, int W, int S, int cap, std::vector<int32_t>& tab, int& G_out) {
    const int64_t n = p->n;
    HostRows hr{p, {}, {}, W};
    if (p->kind == PLAN_CSR) {
        hr.off.resize((size_t)p->n_slices + 1);
        hr.col.resize((size_t)p->sell_entries);
        if (hipMemcpy(hr.off.data(), p->slice_off.ptr, sizeof(int32_t) * hr.off.size(), hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(hr.col.data(), p->col.ptr, sizeof(int32_t) * hr.col.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return false;
    }
    // grid: every column of row m in {m, m +- 1, m +- S1}
    int64_t S1 = 0;
    {
        std::vector<int32_t> c(W);
        for (int64_t m = 0; m < n; ++m) {
            hr.cols(m, c.data());
            for (int j = 0; j < W; ++j) {
                const int64_t d = std::llabs((int64_t)c[j] - m);
                if (d <= 1) continue;
                if (S1 == 0) S1 = d;
                else if (d != S1) return false;
            }
        }
    }
    const bool one_d = S1 == 0;
    if (one_d) S1 = n;
    const int64_t S2 = (n + S1 - 1) / S1;
    // tiles: tw x th cells, Tx x Ty of them, fewest halo cells per tile (a
    // band operator: blocks of kMJOwn consecutive rows)
    int64_t best = -1, Tx = 0, Ty = 0, tw = 0, th = 0;
    if (one_d) {
        Tx = (n + kMJOwn - 1) / kMJOwn;
        Ty = 1;
        tw = kMJOwn;
        th = 1;
        best = Tx <= cap ? 0 : -1;
    }
    for (int64_t tx = 1; !one_d && tx <= std::min<int64_t>(S1, 30); ++tx) {
        const int64_t w = (S1 + tx - 1) / tx;
        if (w > kMJOwn) continue;
        const int64_t hmax = kMJOwn / w;
        const int64_t ty = (S2 + hmax - 1) / hmax;
        const int64_t h = (S2 + ty - 1) / ty;
        if (tx * ty > cap) continue;
        const int64_t cost = (one_d ? 0 : 2 * w) + (S2 > 1 ? 2 * h : 0);
        if (best < 0 || cost < best || (cost == best && tx * ty < Tx * Ty)) {
            best = cost;
            Tx = tx;
            Ty = ty;
            tw = w;
            th = h;
        }
    }
    if (best < 0) return false;
    const int nt = (int)(Tx * Ty);
    const int G = (nt + 7) / 8 * 8;
    if (G > cap) return false;
    auto owner_of = [&](int64_t m, int64_t& li) {
        const int64_t i1 = m % S1, i2 = m / S1;
        const int64_t tx = i1 / tw, ty = i2 / th;
        const int64_t x0 = tx * tw, y0 = ty * th;
        const int64_t w = std::min(tw, S1 - x0);
        li = (i1 - x0) + w * (i2 - y0);
        return (int)(tx + Tx * ty);
    };
    tab.assign((size_t)kMJHdr * G, 0);
    std::vector<std::vector<int32_t>> ring_owner(G);  // owners of each workgroup's ring rows
    std::vector<std::vector<int32_t>> lists(G);
    std::vector<std::array<int32_t, 9>> sizes(G);
    std::vector<int32_t> cbuf(W);
    for (int g = 0; g < G; ++g) {
        std::vector<int32_t>& L = lists[g];
        std::unordered_map<int32_t, int32_t> loc;
        if (g < nt) {
            const int64_t tx = g % Tx, ty = g / Tx, x0 = tx * tw, y0 = ty * th;
            const int64_t w = std::min(tw, S1 - x0), h = std::min(th, S2 - y0);
            for (int64_t iy = 0; iy < h; ++iy)
                for (int64_t ix = 0; ix < w; ++ix) {
                    const int64_t m = x0 + ix + S1 * (y0 + iy);
                    if (m < n) L.push_back((int32_t)m);
                }
        }
        for (size_t i = 0; i < L.size(); ++i) loc.emplace(L[i], (int32_t)i);
        sizes[g][0] = (int32_t)L.size();
        size_t prev = 0;
        for (int j = 1; j <= S; ++j) {
            const size_t end = L.size();
            std::vector<int32_t> fresh;
            // E_j = columns of E_{j-1}; those of E_{j-2} are in E_{j-1} already
            for (size_t r = prev; r < end; ++r) {
                hr.cols(L[r], cbuf.data());
                for (int e = 0; e < W; ++e)
                    if (!loc.count(cbuf[e])) {
                        loc.emplace(cbuf[e], -1);
                        fresh.push_back(cbuf[e]);
                    }
            }
            // ring j in exchange-buffer order
            std::sort(fresh.begin(), fresh.end(), [&](int32_t x, int32_t y) {
                int64_t lx, ly;
                const int ox = owner_of(x, lx), oy = owner_of(y, ly);
                return ox != oy ? ox < oy : lx < ly;
            });
            for (int32_t c : fresh) {
                loc[c] = (int32_t)L.size();
                L.push_back(c);
            }
            prev = j == 1 ? (size_t)sizes[g][0] : (size_t)sizes[g][j - 1];
            sizes[g][j] = (int32_t)L.size();
        }
        const int n0 = sizes[g][0];
        if (sizes[g][S] - n0 > mj_load_cap(S) || sizes[g][S - 1] - n0 > mj_halo_cap(S)) return false;
        for (int32_t i = n0; i < sizes[g][S]; ++i) {
            int64_t li;
            ring_owner[g].push_back(owner_of(L[(size_t)i], li));
        }
        // own rows: gid, local columns; ring rows 1..S-1: gid, local columns;
        // rings 1..S: exchange positions
        int32_t* hd = tab.data() + (size_t)kMJHdr * g;
        for (int j = 0; j <= S; ++j) hd[j] = sizes[g][j];
        hd[kMJHOwn] = (int32_t)tab.size();
        for (int i = 0; i < n0; ++i) tab.push_back(L[(size_t)i]);
        for (int i = 0; i < n0; ++i) {
            hr.cols(L[(size_t)i], cbuf.data());
            for (int e = 0; e < W; ++e) tab.push_back(loc.at(cbuf[e]));
        }
        hd = tab.data() + (size_t)kMJHdr * g;
        hd[kMJHRing] = (int32_t)tab.size();
        const int nh = sizes[g][S - 1] - n0;
        for (int h = 0; h < nh; ++h) tab.push_back(L[(size_t)(n0 + h)]);
        for (int h = 0; h < nh; ++h) {
            hr.cols(L[(size_t)(n0 + h)], cbuf.data());
            for (int e = 0; e < W; ++e) tab.push_back(loc.at(cbuf[e]));
        }
        hd = tab.data() + (size_t)kMJHdr * g;
        hd[kMJHPos] = (int32_t)tab.size();
        {  // rings 1..S by exchange position: positions, then their places after the own rows
            std::vector<std::pair<int32_t, int32_t>> pl;
            for (int32_t i = n0; i < sizes[g][S]; ++i) {
                int64_t li;
                const int o = owner_of(L[(size_t)i], li);
                pl.emplace_back((int32_t)((int64_t)o * kMJOwn + li), i - n0);
            }
            std::sort(pl.begin(), pl.end());
            for (const auto& e : pl) tab.push_back(e.first);
            for (const auto& e : pl) tab.push_back(e.second);
        }
        if (tab.size() >= (size_t)INT32_MAX) return false;
    }
    // neighbour sets: whom I read and who reads me
    std::vector<std::vector<int32_t>> nb(G);
    for (int g = 0; g < G; ++g)
        for (int o : ring_owner[g])
            if (o != g) {
                nb[g].push_back(o);
                nb[o].push_back(g);
            }
    for (int g = 0; g < G; ++g) {
        std::sort(nb[g].begin(), nb[g].end());
        nb[g].erase(std::unique(nb[g].begin(), nb[g].end()), nb[g].end());
        if ((int)nb[g].size() > kMJNb) return false;
        int32_t* hd = tab.data() + (size_t)kMJHdr * g;
        hd[kMJHCount] = (int32_t)nb[g].size();
        for (size_t i = 0; i < nb[g].size(); ++i) hd[kMJHNb + i] = nb[g][i];
    }
    G_out = G;
    return true;
}

static bool persistent_mj_fits_s(mjp_plan* p, int max_open, int S, PersistCfg& cfg);

bool persistent_mj_fits(mjp_plan* p, int max_open, PersistCfg& cfg) {
    for (int S : {8, 4})
        if (persistent_mj_fits_s(p, max_open, S, cfg)) return true;
    return false;
}

static bool persistent_mj_fits_s(mjp_plan* p, int max_open, int S, PersistCfg& cfg) {
    if (max_open > kP2Slots) return false;
    if (p->n >= ((int64_t)1 << 30)) return false;
    if (p->opts.renorm_every % S != 0) return false;  // renormalisation points must end a round
    if (p->opts.barrier_timeout_us < 0) return false;  // the abort-path test uses the two-jump kernel
    if (p->kind == PLAN_STENCIL && stencil_width(p->coef.model) > 5) return false;
    int W = 5;
    if (p->kind == PLAN_CSR) {
        if (p->max_width <= 3) W = 3;
        else if (p->max_width <= 5) W = 5;
        else return false;
    }
    int dev = 0, ncu = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    // Below 16 tiles the one-jump kernel, spread over more workgroups, is used.  At 22 tiles
    // (300 x 300 grid, one time, K = 9344) the tiled sweep takes 1.34 us per jump against 1.97.
    if (p->n < (int64_t)kMJOwn * 16) return false;
    PersistFn f = pick_mj(W, p->kind == PLAN_CSR, S);
    if (!f) return false;
    const size_t lds = mj_lds_for(W, S);
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
        return false;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f), kPThreads, lds) !=
            hipSuccess || per_cu < 1)
        return false;
    const int cap = ncu * per_cu;
    const int key1 = W * 16 + S;
    if (p->mj_key[0] != cap || p->mj_key[1] != key1 || p->mj_key[2] == 0) {
        std::vector<int32_t> tab;
        int G = 0;
        const bool ok = build_mj_table(p, W, S, cap, tab, G);
        p->mj_key[0] = cap;
        p->mj_key[1] = key1;
        p->mj_key[2] = ok ? 1 : 2;
        p->mj_G = G;
        if (ok) {
            if (p->mjtab.reserve(sizeof(int32_t) * tab.size()) != MJP_OK ||
                hipMemcpy(p->mjtab.ptr, tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice) != hipSuccess) {
                p->mj_key[2] = 0;
                return false;
            }
        }
    }
    if (p->mj_key[2] != 1) return false;
    cfg.R = kMJR;
    cfg.W = W;
    cfg.G = p->mj_G;
    cfg.coh = true;
    cfg.jumps = S;
    cfg.fn = reinterpret_cast<const void*>(f);
    return true;
}

bool persistent2_fits(mjp_plan* p, int max_open, PersistCfg& cfg) {
    if (max_open > kP2Slots) return false;
    if (p->n >= ((int64_t)1 << 30)) return false;
    if (p->opts.renorm_every % 2 != 0) return false;  // renormalisation points must end a round
    if (p->kind == PLAN_STENCIL && stencil_width(p->coef.model) > 5) return false;  // halo entries: W <= 5
    int W = 5;
    if (p->kind == PLAN_CSR) {
        if (p->max_width <= 3) W = 3;
        else if (p->max_width <= 5) W = 5;
        else return false;
    }
    int dev = 0, ncu = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    const int64_t need = (p->n + kP2Rows - 1) / kP2Rows;
    const int64_t G = (need + 7) / 8 * 8;
    if (G < ncu / 2) return false;  // too few workgroups to use the chip: the one-jump kernel spreads wider
    const bool force = p->opts.barrier_timeout_us < 0;  // the abort-path test instantiation
    PersistFn f = p->kind == PLAN_CSR ? pick2<true>(W, force) : pick2<false>(W, force);
    if (!f) return false;
    const size_t lds = p2_lds_for(W);
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
        return false;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f), kPThreads, lds) !=
            hipSuccess || per_cu < 1 || G > (int64_t)ncu * per_cu)
        return false;
    if (p->p2_key[0] != (int)G || p->p2_key[1] == 0) {
        std::vector<int32_t> tab;
        const bool ok = build_p2_table(p, (int)G, tab);
        p->p2_key[0] = (int)G;
        p->p2_key[1] = ok ? 1 : 2;
        if (ok) {
            if (p->p2tab.reserve(sizeof(int32_t) * tab.size()) != MJP_OK) {
                p->p2_key[1] = 0;
                return false;
            }
            if (hipMemcpy(p->p2tab.ptr, tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice) != hipSuccess) {
                p->p2_key[1] = 0;
                return false;
            }
        }
    }
    if (p->p2_key[1] != 1) return false;
    cfg.R = kP2R;
    cfg.W = W;
    cfg.G = (int)G;
    cfg.coh = true;
    cfg.jumps = 2;
    cfg.fn = reinterpret_cast<const void*>(f);
    return true;
}

// Tables of the persistent sweep, built once per (plan, G, R) and kept on
// the device:
//  * per-workgroup neighbour interval: the hull of the workgroups owning the
//    columns my rows read and of the workgroups that read my rows.  If some
//    interval spans more than 64 workgroups the sweep uses global barriers
//    only (wait = null).
//  * per-slice bit kSliceLocal: every column the slice reads belongs to its
//    own workgroup (it gathers from the workgroup's LDS copy), decided from
//    the slice's column hull.
static mjp_status build_sweep_tables(mjp_plan* p, const PersistCfg& cfg, const int32_t*& wait_out,
                                     const uint8_t*& sflag_out) {
    wait_out = nullptr;
    sflag_out = nullptr;
    const bool cached = p->wait_key[2] != 0 && p->wait_key[0] == cfg.G && p->wait_key[1] == cfg.R;
    if (cached) {
        if (p->wait_key[2] == 1) wait_out = p->wait.as<int32_t>();
        sflag_out = p->sflag.as<uint8_t>();
        return MJP_OK;
    }
    const int G = cfg.G;
    const int64_t rows_per = (int64_t)kPWaves * cfg.R * 64;
    const int64_t slices_per = rows_per / 64;
    const int64_t n = p->n;
    const int64_t n_slices = (n + 63) / 64;
    // column hull of each slice
    std::vector<int64_t> smin((size_t)n_slices), smax((size_t)n_slices);
    for (int64_t sl = 0; sl < n_slices; ++sl) {
        if (p->kind == PLAN_CSR) {
            smin[(size_t)sl] = p->slice_cmin[(size_t)sl];
            smax[(size_t)sl] = p->slice_cmax[(size_t)sl];
        } else {
            const int64_t reach = stencil_reach(p->coef);
            smin[(size_t)sl] = std::max<int64_t>(0, sl * 64 - reach);
            smax[(size_t)sl] = std::min<int64_t>(n - 1, sl * 64 + 63 + reach);
        }
    }
    // per-slice bits
    std::vector<uint8_t> flag((size_t)n_slices, 0);
    for (int64_t sl = 0; sl < n_slices; ++sl) {
        const int64_t r0 = (sl / slices_per) * rows_per;
        if (smin[(size_t)sl] >= r0 && smax[(size_t)sl] < r0 + rows_per) flag[(size_t)sl] = kSliceLocal;
    }
    mjp_status s = p->sflag.reserve(flag.size());
    if (s) return s;
    MJP_HIP(hipMemcpy(p->sflag.ptr, flag.data(), flag.size(), hipMemcpyHostToDevice));

    std::vector<int32_t> lo(G), hi(G);
    for (int g = 0; g < G; ++g) {
        const int64_t r0 = (int64_t)g * rows_per, r1 = std::min(n, r0 + rows_per);
        if (r0 >= n) { lo[g] = hi[g] = g; continue; }
        int64_t cmin = INT64_MAX, cmax = -1;
        for (int64_t sl = r0 / 64; sl <= (r1 - 1) / 64; ++sl) {
            cmin = std::min(cmin, smin[(size_t)sl]);
            cmax = std::max(cmax, smax[(size_t)sl]);
        }
        lo[g] = (int32_t)std::min<int64_t>(g, cmin / rows_per);
        hi[g] = (int32_t)std::max<int64_t>(g, cmax / rows_per);
    }
    // add the readers of each workgroup's rows
    std::vector<int32_t> wlo(lo), whi(hi);
    for (int g = 0; g < G; ++g)
        for (int h = lo[g]; h <= hi[g]; ++h) {
            wlo[h] = std::min(wlo[h], g);
            whi[h] = std::max(whi[h], g);
        }
    bool ok = true;
    for (int g = 0; g < G && ok; ++g) ok = whi[g] - wlo[g] + 1 <= 64;
    p->wait_key[0] = G;
    p->wait_key[1] = cfg.R;
    sflag_out = p->sflag.as<uint8_t>();
    if (!ok) {
        p->wait_key[2] = 2;
        return MJP_OK;
    }
    std::vector<int32_t> tab(2 * (size_t)G);
    for (int g = 0; g < G; ++g) {
        tab[2 * (size_t)g] = wlo[g];
        tab[2 * (size_t)g + 1] = whi[g];
    }
    if ((s = p->wait.reserve(sizeof(int32_t) * tab.size()))) return s;
    MJP_HIP(hipMemcpy(p->wait.ptr, tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice));
    p->wait_key[2] = 1;
    wait_out = p->wait.as<int32_t>();
    return MJP_OK;
}

mjp_status launch_persistent(mjp_plan* p, const PersistCfg& cfg, const float* rho0, const AllTimes& at,
                             const std::vector<int>& slot, float* out, hipStream_t st) {
    const int64_t n = p->n;
    // the multi-jump kernel's exchange buffers hold kMJOwn rows per workgroup
    const int64_t nbuf = cfg.jumps >= 4 ? std::max<int64_t>(n, (int64_t)cfg.G * kMJOwn) : n;
    mjp_status s;
    if ((s = p->rho[0].reserve(sizeof(float) * nbuf)) || (s = p->rho[1].reserve(sizeof(float) * nbuf)) ||
        (s = p->sync.reserve(sizeof(unsigned) * (kBarWords + 32 * (size_t)cfg.G) + sizeof(double) * 3 * (size_t)cfg.G)))
        return s;
    unsigned* bar = p->sync.as<unsigned>();
    unsigned* wflag = bar + kBarWords;
    double* pmass = reinterpret_cast<double*>(wflag + 32 * (size_t)cfg.G);
    const int32_t* wait = nullptr;
    const uint8_t* sflag = nullptr;
    if (cfg.jumps == 1 && (s = build_sweep_tables(p, cfg, wait, sflag))) return s;
    double* mass_out = p->scal.as<double>() + S_MASS0;  // [S_MASS0], [S_MASSK]
    PersistArgs a{};
    a.slice_off = p->slice_off.as<int32_t>();
    a.col = p->col.as<int32_t>();
    a.val = p->val.as<float>();
    a.dlo = p->dlo.as<float>();
    a.cf = p->coef;
    a.rho0 = rho0;
    a.buf0 = p->rho[0].as<float>();
    a.buf1 = p->rho[1].as<float>();
    a.out = out;
    a.wtab = p->wtab.as<double>();
    a.pmass = pmass;
    a.bar = bar;
    a.wflag = wflag;
    a.wait = wait;
    a.sflag = sflag;
    a.p2 = cfg.jumps == 2 ? p->p2tab.as<int32_t>() : (cfg.jumps >= 4 ? p->mjtab.as<int32_t>() : nullptr);
    a.flags = reinterpret_cast<unsigned*>(p->scal.as<double>() + S_FLAGS);
    a.mass_out = mass_out;
    a.n = n;
    a.n_slices = (int32_t)((n + 63) / 64);
    a.Kmax = 0;
    for (int j = 0; j < at.n; ++j) a.Kmax = std::max(a.Kmax, at.tp[j].K);
    a.renorm_every = p->opts.renorm_every;
    a.G = cfg.G;
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device) != hipSuccess || khz <= 0)
            khz = 100000;
        const int32_t us = p->opts.barrier_timeout_us;  // <= 0: 2 s (< 0 selects the forcing two-jump kernel)
        a.timeout_ticks = us <= 0 ? (uint64_t)khz * 1000ull * 2ull : (uint64_t)khz * (uint64_t)us / 1000ull;
    }
    a.at = at;
    for (int j = 0; j < at.n; ++j) a.slot[j] = slot[(size_t)j];
    const int nzero = kBarWords + 32 * cfg.G;
    hipLaunchKernelGGL(k_zero_u32, dim3((nzero + 255) / 256), dim3(256), 0, st, bar, nzero);
    void* args[] = {&a};
    const size_t lds = cfg.jumps == 2 ? p2_lds_for(cfg.W) : (cfg.jumps >= 4 ? mj_lds_for(cfg.W, cfg.jumps) : 0);
    MJP_HIP(hipLaunchCooperativeKernel(cfg.fn, dim3(cfg.G), dim3(kPThreads), args, lds, st));
    return MJP_OK;
}

// Times `rounds` exchange-only rounds on the two-jump sweep's launch
// configuration for this plan (HIP events on st); false if the plan's sweep
// does not run the two-jump kernel.
mjp_status probe_exchange(mjp_plan* p, int rounds, hipStream_t st, float* ms_out, int* jumps_out) {
    PersistCfg cfg;
    const bool multi = (p->opts.variant == MJP_VARIANT_AUTO || p->opts.variant == MJP_VARIANT_PERSISTENT) &&
                       persistent_mj_fits(p, 1, cfg);
    MJP_CHECK(multi || persistent2_fits(p, 1, cfg), MJP_E_UNSUPPORTED,
              "the plan's sweep synchronises every jump (no two-jump or tiled kernel)");
    *jumps_out = cfg.jumps;
    const int64_t n = p->n;
    // the multi-jump kernel's exchange buffers hold kMJOwn rows per workgroup
    const int64_t nbuf = cfg.jumps >= 4 ? std::max<int64_t>(n, (int64_t)cfg.G * kMJOwn) : n;
    mjp_status s;
    if ((s = p->rho[0].reserve(sizeof(float) * nbuf)) || (s = p->rho[1].reserve(sizeof(float) * nbuf)) ||
        (s = p->sync.reserve(sizeof(unsigned) * (kBarWords + 32 * (size_t)cfg.G) + sizeof(double) * 3 * (size_t)cfg.G)) ||
        (s = p->scal.reserve(sizeof(double) * S_COUNT)))
        return s;
    unsigned* bar = p->sync.as<unsigned>();
    PersistArgs a{};
    a.rho0 = p->rho[1].as<float>();  // any defined vector: the probe only copies it around
    a.buf0 = p->rho[0].as<float>();
    a.buf1 = p->rho[1].as<float>();
    a.bar = bar;
    a.wflag = bar + kBarWords;
    a.p2 = multi ? p->mjtab.as<int32_t>() : p->p2tab.as<int32_t>();
    a.flags = reinterpret_cast<unsigned*>(p->scal.as<double>() + S_FLAGS);
    a.n = n;
    a.G = cfg.G;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device) != hipSuccess || khz <= 0) khz = 100000;
    a.timeout_ticks = (uint64_t)khz * 1000ull * 2ull;
    const void* fn = !multi ? reinterpret_cast<const void*>(k_exchange_probe<false>)
                     : cfg.jumps == 8 ? reinterpret_cast<const void*>(k_exchange_probe_mj<8>)
                                      : reinterpret_cast<const void*>(k_exchange_probe_mj<4>);
    const size_t lds = !multi ? sizeof(float) * kP2X2 : mj_probe_lds_bytes(cfg.jumps);
    MJP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int nzero = kBarWords + 32 * cfg.G;
    hipEvent_t e0, e1;
    MJP_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MJP_E_DEVICE, "hipEventCreate failed");
    }
    hipError_t he = hipSuccess;
    float ms = 0.f;
    for (int rep = 0; rep < 2 && he == hipSuccess; ++rep) {  // the first run warms up
        hipLaunchKernelGGL(k_zero_u32, dim3((nzero + 255) / 256), dim3(256), 0, st, bar, nzero);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(a.flags), 2);
        he = hipEventRecord(e0, st);
        void* args[] = {&a, &rounds};
        if (he == hipSuccess) he = hipLaunchCooperativeKernel(fn, dim3(cfg.G), dim3(kPThreads), args, lds, st);
        if (he == hipSuccess) he = hipEventRecord(e1, st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    }
    unsigned fl = 0;
    if (he == hipSuccess) he = hipMemcpy(&fl, a.flags, sizeof(unsigned), hipMemcpyDeviceToHost);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    MJP_CHECK(he == hipSuccess, MJP_E_DEVICE, "exchange probe failed: %s", hipGetErrorString(he));
    MJP_CHECK(!(fl & kFlagBarrierTimeout), MJP_E_DEVICE, "exchange probe: a wait missed its deadline");
    *ms_out = ms;
    return MJP_OK;
}

}  // namespace mjp
