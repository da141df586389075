// Device-side helpers shared by the ORBGRAND kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ORBG_WAVE 64
#define ORBG_RANK_SLOTS 256   // LDS slots per wave for permuted columns: rank 0 is the zero column
#define ORBG_ENTRY_RANKS 16   // ranks held by one 16-byte schedule entry (u8 each, 0 = unused)

namespace orbg {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Orders this wave's LDS traffic: every lane's earlier LDS writes are visible to
// every lane's later LDS reads (waits for the LDS queue, keeps the compiler
// from moving accesses across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// XOR of one 32-bit value over the 16 lanes of each DPP row (every lane of the
// row receives it): quad swaps, half-row mirror, row mirror.  All lanes active.
__device__ __forceinline__ uint32_t row_xor16(uint32_t v)
{
    v ^= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v ^= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v ^= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v ^= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    return v;
}

// XOR of a u64 over the whole wave, returned wave-uniform.  All lanes active.
__device__ __forceinline__ uint64_t wave_xor_reduce(uint64_t v)
{
    const uint32_t lo = row_xor16((uint32_t)v), hi = row_xor16((uint32_t)(v >> 32));
    const uint32_t l = __builtin_amdgcn_readlane(lo, 0) ^ __builtin_amdgcn_readlane(lo, 16) ^
                       __builtin_amdgcn_readlane(lo, 32) ^ __builtin_amdgcn_readlane(lo, 48);
    const uint32_t h = __builtin_amdgcn_readlane(hi, 0) ^ __builtin_amdgcn_readlane(hi, 16) ^
                       __builtin_amdgcn_readlane(hi, 32) ^ __builtin_amdgcn_readlane(hi, 48);
    return ((uint64_t)h << 32) | l;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Ascending bitonic sort of 64*NK u64 keys held NK per lane.  Element e lives
// in lane e / NK, register e % NK, so distances below NK are exchanged inside a
// lane and larger ones across lanes (lane distance d / NK).  Keys must be
// distinct except for padding.  A compare-exchange is one 64-bit compare, a
// lane-mask XOR with the stage's direction and two selects.
template <int NK, typename KEY = uint64_t>
__device__ __forceinline__ void bitonic_sort(KEY (&key)[NK])
{
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= ORBG_WAVE * NK; size <<= 1) {
#pragma unroll
        for (int d = size >> 1; d > 0; d >>= 1) {
            if (d < NK) {
#pragma unroll
                for (int j = 0; j < NK; ++j) {
                    if ((j & d) == 0) {
                        // ascending iff bit `size` of e = lane * NK + j is clear
                        const bool desc = ((lane * NK + j) & size) != 0;
                        const KEY a = key[j], b = key[j | d];
                        const bool sw = (a > b) != desc;
                        key[j] = sw ? b : a;
                        key[j | d] = sw ? a : b;
                    }
                }
            } else {
                const int ld = d / NK;
                // the lower lane of a pair keeps the minimum in ascending runs
                const bool keep_min = ((lane & ld) == 0) == (((lane * NK) & size) == 0);
#pragma unroll
                for (int j = 0; j < NK; ++j) {
                    const KEY p = __shfl_xor(key[j], ld, ORBG_WAVE);
                    const bool take_p = (p < key[j]) == keep_min;
                    key[j] = take_p ? p : key[j];
                }
            }
        }
    }
}

}  // namespace orbg
