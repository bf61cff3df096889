// Grid-wide synchronisation of a cooperative launch (every workgroup
// co-resident), shared by the persistent R-MJP sweep and the fused Krylov
// step: the publishing/acquiring halves of a synchronisation point under the
// two memory protocols, and a two-level grid barrier with a wall-clock
// deadline.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mjp {

// bit of a flags word raised when a grid barrier timed out
constexpr unsigned kFlagBarrierTimeout = 0x80000000u;

// A waiting wave re-reads what it waits for every spin, but the abort word
// (another device-scope round trip) and its wall-clock deadline only every
// kAbortCheckEvery spins, so a spin costs one memory round trip.
// FORCE (a separate instantiation, used only when the host asks for it):
// a wait whose first read finds the word not yet set gives up at once,
// raising the abort flag -- the host's way to exercise the abort path.
constexpr unsigned kAbortCheckEvery = 16;

__device__ __forceinline__ int logical_block(int G) {
    // workgroups are dispatched round-robin over the 8 XCDs; renumber so
    // that XCD x runs logical blocks [x*G/8, (x+1)*G/8)
    const int b = blockIdx.x;
    return (b & 7) * (G >> 3) + (b >> 3);
}

// Publishing side of a synchronisation point.  COH: every wave waits until
// its own loads and stores have completed (device-scope stores are then
// visible to every XCD, and the loads of the buffer about to be overwritten
// have returned).  Fenced: the release fence is issued by the publishing
// thread after the workgroup barrier.
template <bool COH>
__device__ __forceinline__ void drain_wave() {
    if constexpr (COH) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}
template <bool COH>
__device__ __forceinline__ void release_agent() {
    if constexpr (!COH) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}
template <bool COH>
__device__ __forceinline__ void acquire_agent() {
    if constexpr (!COH) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Iterate accesses under either protocol: raw buffer loads and stores at a
// 32-bit byte offset from a uniform descriptor (one offset register per
// gather instead of a 64-bit address pair).  The descriptor's range is the
// vector's n*4 bytes, so an access past the end reads 0 or is dropped.  COH
// sets the device-scope cache policy (the SC1 bit of the instruction's
// cache-policy operand on this architecture family), which is what the
// compiler emits for an agent-scope relaxed atomic load or store.
constexpr int kCpolSC1 = 16;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t iter_rsrc(const float* p, int64_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, (int)(uint32_t)(4 * n), kRsrcWord3);
}
// (the b32 builtins move 32-bit integers: the float travels as its bits)
template <bool COH>
__device__ __forceinline__ float ld_iter(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, COH ? kCpolSC1 : 0));
}
template <bool COH>
__device__ __forceinline__ void st_iter(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, COH ? kCpolSC1 : 0);
}

// Barrier words (unsigned), each on its own 256-byte line:
//   [x*64]      arrival counter of XCD group x (x < 8)
//   [8*64]      arrival counter of the group leaders
//   [(9+x)*64]  release epoch as seen by group x
constexpr int kBarWords = 17 * 64;

// Two-level grid barrier.  Each workgroup arrives on its XCD group's
// counter (relaxed add after the publishing step); the last arrival of a
// group arrives on the top counter; the last of those publishes the epoch to
// the eight group words, which each group polls with relaxed loads.  In the
// fenced protocol every hand-off re-fences (acquire then release), so each
// arrival's writes happen-before every reader's acquire; in the COH protocol
// every arrival's device-scope writes were complete before it arrived, so
// the hand-offs need no fences.  Spreading the arrivals over 8 counters
// removes most of the contention of a single counter hit by every
// workgroup.  Returns false if the sweep was aborted (a wait exceeded its
// wall-clock deadline somewhere); every workgroup then leaves the kernel.
template <bool COH, bool FORCE = false>
__device__ __forceinline__ bool grid_barrier(unsigned* w, unsigned epoch, int g, int G, unsigned* flags,
                                             uint64_t timeout_ticks) {
    __shared__ int aborted;
    drain_wave<COH>();
    __syncthreads();
    if (G == 1) return true;  // a single workgroup: its own barrier is the grid barrier
    if (threadIdx.x == 0) {
        aborted = 0;
        const int per = G >> 3, grp = g / per;
        release_agent<COH>();
        const unsigned old = __hip_atomic_fetch_add(&w[grp * 64], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == epoch * (unsigned)per - 1u) {
            acquire_agent<COH>();
            release_agent<COH>();
            const unsigned o2 = __hip_atomic_fetch_add(&w[8 * 64], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (o2 == epoch * 8u - 1u) {
                acquire_agent<COH>();
                release_agent<COH>();
                for (int x = 0; x < 8; ++x)
                    __hip_atomic_store(&w[(9 + x) * 64], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if constexpr (FORCE) {
            if (__hip_atomic_load(&w[(9 + grp) * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
                __hip_atomic_fetch_or(flags, kFlagBarrierTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                aborted = 1;
            }
        } else {
            const uint64_t t0 = wall_clock64();
            unsigned spins = 0;
            while (__hip_atomic_load(&w[(9 + grp) * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins % kAbortCheckEvery != 0) continue;
                if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagBarrierTimeout) {
                    aborted = 1;
                    break;
                }
                if (wall_clock64() - t0 > timeout_ticks) {
                    __hip_atomic_fetch_or(flags, kFlagBarrierTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    aborted = 1;
                    break;
                }
            }
        }
        acquire_agent<COH>();
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(aborted) == 0;  // uniform: every thread read the same word
}

}  // namespace mjp
