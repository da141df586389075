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

// Value of lane (lane XOR LD) for a wave-constant distance LD, all lanes active:
// quad permutes for 1 and 2, a half-row mirror composed with a quad reversal for
// 4 (7 - (i ^ 3) = i ^ 4 inside each group of 8), a half-row rotation for 8, an
// LDS-crossbar swizzle (xor mask 16 inside 32 lanes) for 16 and a bpermute for 32.
template <int LD>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v)
{
    static_assert(LD == 1 || LD == 2 || LD == 4 || LD == 8 || LD == 16 || LD == 32, "lane distance");
    if constexpr (LD == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    } else if constexpr (LD == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    } else if constexpr (LD == 4) {
        const int m = __builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);     // row_half_mirror
        return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false);        // quad_perm [3,2,1,0]
    } else if constexpr (LD == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else if constexpr (LD == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);               // and 0x1f, xor 0x10
    } else {
        return (uint32_t)__shfl_xor((int)v, 32, 64);
    }
}

// Lane masks of the bitonic network (compile-time constants): in a cross-lane
// substep of stage `size` at lane distance ld, the lanes that keep the smaller
// key; in an in-lane substep, the lanes whose register j runs descending.
constexpr uint64_t keep_min_mask(int nk, int size, int ld)
{
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l)
        if (((l & ld) == 0) == (((l * nk) & size) == 0)) m |= 1ull << l;
    return m;
}
constexpr uint64_t desc_mask(int nk, int size, int j)
{
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l)
        if (((l * nk + j) & size) != 0) m |= 1ull << l;
    return m;
}

// Per-lane bit of a constant lane mask.  The two scalar moves are written out
// so that the constant is made where it is used: the compiler would otherwise
// hoist it out of the block loop, spill it and reload it with vector
// instructions.
template <uint64_t M>
__device__ __forceinline__ bool lane_bit()
{
    uint32_t lo, hi;
    asm volatile("s_mov_b32 %0, %2\n\ts_mov_b32 %1, %3"
                 : "=s"(lo), "=s"(hi)
                 : "i"((int32_t)(uint32_t)M), "i"((int32_t)(uint32_t)(M >> 32)));
    return __builtin_amdgcn_inverse_ballot_w64(((uint64_t)hi << 32) | lo);
}

// One in-lane compare-exchange of registers J and J | D (for every J without bit D).
template <int NK, int SIZE, int D, int J>
__device__ __forceinline__ void bitonic_inlane32(uint32_t (&key)[NK])
{
    if constexpr (J < NK) {
        if constexpr ((J & D) == 0) {
            const bool desc = lane_bit<desc_mask(NK, SIZE, J)>();
            const uint32_t a = key[J], b = key[J | D];
            const bool sw = (a > b) != desc;
            key[J] = sw ? b : a;
            key[J | D] = sw ? a : b;
        }
        bitonic_inlane32<NK, SIZE, D, J + 1>(key);
    }
}

// Substeps D, D/2, ..., 1 of stage SIZE.
template <int NK, int SIZE, int D>
__device__ __forceinline__ void bitonic_step32(uint32_t (&key)[NK])
{
    if constexpr (D >= NK) {
        constexpr int LD = D / NK;
        const bool keep_min = lane_bit<keep_min_mask(NK, SIZE, LD)>();
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const uint32_t p = lane_xor<LD>(key[j]);
            const bool take_p = (p < key[j]) == keep_min;
            key[j] = take_p ? p : key[j];
        }
    } else {
        bitonic_inlane32<NK, SIZE, D, 0>(key);
    }
    if constexpr (D > 1) bitonic_step32<NK, SIZE, D / 2>(key);
}

template <int NK, int SIZE, int MAXSIZE>
__device__ __forceinline__ void bitonic_stage32(uint32_t (&key)[NK])
{
    bitonic_step32<NK, SIZE, SIZE / 2>(key);
    if constexpr (SIZE < MAXSIZE) bitonic_stage32<NK, SIZE * 2, MAXSIZE>(key);
}

// Ascending bitonic sort of 64*NK distinct u32 keys, element e = lane * NK + j
// in register j of its lane (same network as bitonic_sort), with the lane
// exchanges of lane_xor (no LDS traffic below lane distance 16) and the stage
// directions as constant scalar lane masks: a compare-exchange is a lane
// exchange, one compare and one select.
template <int NK>
__device__ __forceinline__ void bitonic_sort32(uint32_t (&key)[NK])
{
    bitonic_stage32<NK, 2, ORBG_WAVE * NK>(key);
}

// One key per lane, the first log2(GROUP) stages of the same network: lanes
// 0..GROUP-1 end sorted ascending (the following groups alternate direction).
template <int GROUP>
__device__ __forceinline__ void bitonic_sort32_groups(uint32_t (&key)[1])
{
    bitonic_stage32<1, 2, GROUP>(key);
}

}  // namespace orbg
