// Device-side helpers shared by the HIP kernels of libhlf (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hlf.h"

namespace hlf {

constexpr int kWave = 64;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// Four dwords, for 16-byte loads and stores (nontemporal builtins accept it).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Output function of SplitMix64 (Stafford's Mix13), used for the set hash and
// the sampling coefficient stream.
__device__ __forceinline__ uint64_t mix13(uint64_t x) {
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

// mix13 without its first step x ^= x >> 30.  That step is linear over GF(2),
// so for x = a ^ b it equals (a ^ (a >> 30)) ^ (b ^ (b >> 30)); callers that
// split x into a per-lane and a per-tile part pre-apply it to each part.
__device__ __forceinline__ uint64_t mix13_tail(uint64_t x) {
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

__device__ __forceinline__ uint64_t mix13_head(uint64_t x) { return x ^ (x >> 30); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// A value that is the same on every lane, moved to scalar registers.
// XOR of v over lanes 0..7 of a wave, returned to every lane.  Needs all
// lanes active.  Three DPP row_shr steps leave the XOR of lanes 0..7 in lane
// 7 (a disabled source lane contributes the identity 0 through `old`).
__device__ __forceinline__ uint32_t xor_lanes0to7(uint32_t v) {
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
    v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 7);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ uint64_t wave_xor_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v ^= __shfl_xor(v, off, kWave);
    return v;
}

// 64x64 bit transpose across one wavefront: lane l holds row l (bit c =
// column c) and gets column l (bit r = row r).  Step j swaps, between lanes l
// and l ^ j, the bits whose row and column indices differ in bit j, so after
// the six steps bit (r, c) sits at (r ^ d, c ^ d), d = r ^ c, i.e. at (c, r).
// Needs all lanes active.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
#pragma unroll
    for (int step = 5; step >= 0; --step) {
        const int j = 1 << step;
        const uint64_t m = j == 32 ? 0x00000000FFFFFFFFull
                         : j == 16 ? 0x0000FFFF0000FFFFull
                         : j == 8  ? 0x00FF00FF00FF00FFull
                         : j == 4  ? 0x0F0F0F0F0F0F0F0Full
                         : j == 2  ? 0x3333333333333333ull
                                   : 0x5555555555555555ull;
        const uint64_t y = __shfl_xor(x, j, kWave);
        x = (lane & j) ? ((x & ~m) | ((y & ~m) >> j)) : ((x & m) | ((y & m) << j));
    }
    return x;
}

// Orders the LDS accesses of one wavefront around this point (waits for its
// outstanding LDS operations; no other wave is involved).  Used by code that
// runs on a single wave of a larger workgroup.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Mask of the valid bits of the last word of an n-bit vector (all ones when
// n is a multiple of 64).
__device__ __forceinline__ uint64_t last_word_mask(int n) {
    int rem = n & 63;
    return rem ? ((1ull << rem) - 1) : ~0ull;
}

}  // namespace hlf
