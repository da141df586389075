// Basic ORBGRAND decode kernels for gfx950 (one wave64 per received block).
//
// Per block (Algorithm 1 with the basic ORBGRAND generator):
//   1. stage: the block's LLR row is read coalesced (lane l holds elements
//      l, l+64, ...); the code's packed parity-check columns (u64, bit r = H[r][i])
//      sit in LDS, shared by the workgroup;
//   2. hard decision y_i = [LLR_i > 0] (Sec. III-A) and base syndrome
//      s0 = XOR of the columns with y_i = 1; s0 == 0 means query 1 (no flip) is
//      a code-book member and nothing else is needed;
//   3. rank: keys (IEEE bits of |LLR_i|) << 32 | i sorted ascending by a
//      register bitonic network (stable by index, the permutation of Sec. III-A);
//      h_j = column of the j-th least reliable bit is written to LDS for the
//      ranks the schedule can reach, and T[m] = s0 XOR (XOR of h_j over the bits
//      of m) for all 256 subsets m of ranks 1..8;
//   4. search: the wave tests 64 consecutive schedule entries per step, lane l
//      taking entry 64t + l; its syndrome is T[low mask] XOR h_{r} over the
//      entry's ranks above 8 (the parity-check product is linear, Sec. I), and a
//      ballot of "syndrome == 0" gives the lowest-index hit, so the result is
//      the first code-book member in schedule order whatever the timing.  The
//      next step's entries are loaded while the current step is tested;
//   5. output: codeword in received order, queries used, abandon flag (budget
//      exhausted without a hit, Sec. IV-A).
//
// Waves are persistent: each takes chunks of blocks from an atomic counter, so
// blocks needing very different numbers of queries balance across the chip.
// With a batch order (learned proposal) step t < 64 tests batch order[t] of the
// schedule instead of batch t; from step 64 on the plain order continues.
#include "orbg_device.h"
#include "orbg_internal.h"
#include "orbg_kernels.h"

namespace orbg {

// Per-wave LDS: the syndrome type S is u32 when n - k <= 32, else u64.
template <typename S>
struct WaveLds {
    S T[256];                           // s0 ^ syndromes of the subsets of ranks 1..8
    S h[ORBG_RANK_SLOTS];               // h[r] = column of rank r (h[0] = 0)
    uint16_t pi[ORBG_RANK_SLOTS];       // pi[r] = received index of rank r
};

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

template <int NK>
__device__ __forceinline__ void load_row(const float* __restrict__ llr_row, int n, float (&x)[NK])
{
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane_id();
        x[j] = (i < n) ? llr_row[i] : 0.0f;
    }
}

// Mask of the lowest `cnt` lanes.
__device__ __forceinline__ uint64_t low_lanes(uint32_t cnt) { return cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull); }

// Batch tested at step t: the block's order for the first 64 steps (values
// taken modulo 64), the plain order afterwards.
template <bool ORDERED>
__device__ __forceinline__ uint32_t batch_at(const uint8_t* __restrict__ order_row, uint32_t t)
{
    if (!ORDERED || t >= 64) return t;
    return uniform_u32(order_row[t]) & 63u;
}

template <typename S>
__device__ __forceinline__ S wave_xor_reduce_s(S v);
template <>
__device__ __forceinline__ uint32_t wave_xor_reduce_s<uint32_t>(uint32_t v)
{
    const uint32_t r = row_xor16(v);
    return __builtin_amdgcn_readlane(r, 0) ^ __builtin_amdgcn_readlane(r, 16) ^
           __builtin_amdgcn_readlane(r, 32) ^ __builtin_amdgcn_readlane(r, 48);
}
template <>
__device__ __forceinline__ uint64_t wave_xor_reduce_s<uint64_t>(uint64_t v) { return wave_xor_reduce(v); }

template <int NK, bool ORDERED, typename S>
__device__ __forceinline__ void decode_block(
    const float (&x)[NK], int n, const S* __restrict__ s_cols, WaveLds<S>& L,
    const uint2* __restrict__ sched, const uint32_t* __restrict__ bh, uint32_t slen, int rdepth,
    uint32_t budget, const uint8_t* __restrict__ order_row,
    uint8_t* __restrict__ cw_row, uint64_t* __restrict__ q_out, uint8_t* __restrict__ ab_out)
{
    const int lane = lane_id();

    // 1-2. hard decision, base syndrome (the row was staged by the caller)
    S acc = 0;
    bool ybit[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane;
        ybit[j] = (i < n) && (x[j] > 0.0f);
        acc ^= ybit[j] ? s_cols[i] : (S)0;
    }
    const S s0 = wave_xor_reduce_s<S>(acc);

    bool found = false;
    uint32_t q = budget;
    uint32_t win_lo = 0, win_hi = 0;     // winning entry (wave-uniform)

    if (!ORDERED && s0 == 0) {
        found = true;
        q = 1;
    } else {
        // 3. rank
        uint64_t key[NK];
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int i = j * ORBG_WAVE + lane;
            key[j] = (i < n) ? (((uint64_t)(__float_as_uint(x[j]) & 0x7fffffffu) << 32) | (uint32_t)i)
                             : ~0ull;
        }
        bitonic_sort<NK>(key);
        wave_lds_sync();
        if (lane == 0) { L.h[0] = 0; L.pi[0] = 0; }
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int e = lane * NK + j;          // rank e + 1
            if (e < rdepth) {
                const uint32_t idx = (uint32_t)key[j];
                L.h[e + 1] = s_cols[idx];
                L.pi[e + 1] = (uint16_t)idx;
            } else if (e < ORBG_LOW_RANKS) {
                L.h[e + 1] = 0;                   // ranks beyond n (tiny codes)
            }
        }
        wave_lds_sync();
        S a = s0;
#pragma unroll
        for (int b = 0; b < 6; ++b) a ^= ((lane >> b) & 1) ? L.h[b + 1] : (S)0;
        const S h7 = L.h[7], h8 = L.h[8];
        L.T[lane] = a;
        L.T[lane + 64] = a ^ h7;
        L.T[lane + 128] = a ^ h8;
        L.T[lane + 192] = a ^ h7 ^ h8;
        wave_lds_sync();

        // 4. search.  Step t tests batch bt; lane l takes schedule entry 64 bt + l,
        // which is query number 64 t + l + 1.  Lanes past the budget or the
        // schedule read a valid entry and are masked out of the ballot.
        // Indices fit 32 bits (budget, schedule length <= 2^22).
        uint32_t t = 0;
        uint32_t bt = batch_at<ORDERED>(order_row, 0);
        uint64_t vmask = low_lanes(min(budget, slen - bt * ORBG_WAVE));
        uint2 ent = sched[min(bt * ORBG_WAVE + lane, slen - 1)];
        uint32_t nh = bh[bt];
        for (;;) {
            const uint32_t t1 = t + 1;
            const uint32_t b1 = batch_at<ORDERED>(order_row, t1);
            const bool has_next = (t1 * ORBG_WAVE < budget) && (b1 * ORBG_WAVE < slen);
            uint2 ent1 = make_uint2(0u, 0u);
            uint32_t nh1 = 0;
            uint64_t vmask1 = 0;
            if (has_next) {
                ent1 = sched[min(b1 * ORBG_WAVE + lane, slen - 1)];
                nh1 = bh[b1];
                vmask1 = low_lanes(min(budget - t1 * ORBG_WAVE, slen - b1 * ORBG_WAVE));
            }
            // all lookups issued before the first XOR
            const S v0 = L.T[ent.x & 0xffu];
            S v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0, v6 = 0, v7 = 0;
            if (nh >= 1) v1 = L.h[(ent.x >> 8) & 0xffu];
            if (nh >= 2) v2 = L.h[(ent.x >> 16) & 0xffu];
            if (nh >= 3) v3 = L.h[ent.x >> 24];
            if (nh >= 4) v4 = L.h[ent.y & 0xffu];
            if (nh >= 5) v5 = L.h[(ent.y >> 8) & 0xffu];
            if (nh >= 6) v6 = L.h[(ent.y >> 16) & 0xffu];
            if (nh >= 7) v7 = L.h[ent.y >> 24];
            const S syn = v0 ^ v1 ^ v2 ^ v3 ^ v4 ^ v5 ^ v6 ^ v7;
            const uint64_t hits = ballot(syn == 0) & vmask;
            if (hits) {
                const int wl = __builtin_ctzll(hits);
                found = true;
                q = t * ORBG_WAVE + wl + 1;
                win_lo = __builtin_amdgcn_readlane(ent.x, wl);
                win_hi = __builtin_amdgcn_readlane(ent.y, wl);
                break;
            }
            if (!has_next) break;
            t = t1; ent = ent1; nh = nh1; vmask = vmask1;
        }
    }

    // 5. output: the hard decision with the winning pattern's positions flipped
    if ((win_lo | win_hi) == 0) {
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int i = j * ORBG_WAVE + lane;
            if (i < n) cw_row[i] = ybit[j] ? 1 : 0;
        }
    } else {
        int flip_pos[ORBG_LOW_RANKS + ORBG_HIGH_SLOTS];
#pragma unroll
        for (int u = 0; u < ORBG_LOW_RANKS; ++u)
            flip_pos[u] = ((win_lo >> u) & 1u) ? (int)L.pi[u + 1] : -1;
#pragma unroll
        for (int u = 1; u <= ORBG_HIGH_SLOTS; ++u) {
            const uint32_t r = (u < 4) ? ((win_lo >> (8 * u)) & 0xffu) : ((win_hi >> (8 * (u - 4))) & 0xffu);
            flip_pos[ORBG_LOW_RANKS + u - 1] = r ? (int)L.pi[r] : -1;
        }
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int i = j * ORBG_WAVE + lane;
            if (i < n) {
                bool b = ybit[j];
#pragma unroll
                for (int u = 0; u < ORBG_LOW_RANKS + ORBG_HIGH_SLOTS; ++u) b ^= (flip_pos[u] == i);
                cw_row[i] = b ? 1 : 0;
            }
        }
    }
    if (lane == 0) {
        *q_out = found ? q : budget;
        *ab_out = found ? 0 : 1;
    }
    wave_lds_sync();
}

// One wave per workgroup, so the wave's LDS tables sit at fixed addresses.
template <int NK, bool ORDERED, typename S>
__global__ void __launch_bounds__(ORBG_WAVE)
decode_kernel(const float* __restrict__ llr, int64_t nblocks, int n,
              const uint64_t* __restrict__ cols,
              const uint2* __restrict__ sched, const uint32_t* __restrict__ bh, uint32_t slen, int rdepth,
              uint32_t budget, const uint8_t* __restrict__ order,
              uint8_t* __restrict__ cw, uint64_t* __restrict__ queries, uint8_t* __restrict__ abandoned,
              unsigned long long* __restrict__ work, int chunk)
{
    __shared__ S s_cols[ORBG_WAVE * NK];
    __shared__ WaveLds<S> L;
    for (int i = threadIdx.x; i < n; i += ORBG_WAVE) s_cols[i] = (S)cols[i];
    wave_lds_sync();
    const int lane = lane_id();

    // XCD-aware work split: workgroups are dealt round-robin to the 8 XCDs, so
    // workgroup w works first on slice w % 8 of the blocks through that slice's
    // counter (an atomic in the XCD's own L2), then helps the other slices.
    const int home = (int)(blockIdx.x % ORBG_XCDS);
    for (int k = 0; k < ORBG_XCDS; ++k) {
        const int xs = (home + k) % ORBG_XCDS;
        const int64_t lo = nblocks * xs / ORBG_XCDS, hi = nblocks * (xs + 1) / ORBG_XCDS;
        unsigned long long* ctr = work + xs * ORBG_COUNTER_STRIDE;
        unsigned long long c0 = 0;
        if (lane == 0) c0 = atomicAdd(ctr, (unsigned long long)chunk);
        int64_t b0 = lo + (int64_t)__shfl(c0, 0, ORBG_WAVE);
        while (b0 < hi) {
            unsigned long long c1 = 0;
            if (lane == 0) c1 = atomicAdd(ctr, (unsigned long long)chunk);   // in flight meanwhile
            const int64_t end = (b0 + chunk < hi) ? b0 + chunk : hi;
            float x[NK];
            load_row<NK>(llr + b0 * n, n, x);
            for (int64_t b = b0; b < end; ++b) {
                float xn[NK];
                if (b + 1 < end) load_row<NK>(llr + (b + 1) * n, n, xn);   // next row in flight
                decode_block<NK, ORDERED, S>(x, n, s_cols, L, sched, bh, slen, rdepth, budget,
                                             ORDERED ? order + b * 64 : nullptr, cw + b * n, queries + b,
                                             abandoned + b);
#pragma unroll
                for (int j = 0; j < NK; ++j) x[j] = xn[j];
            }
            b0 = lo + (int64_t)__shfl(c1, 0, ORBG_WAVE);
        }
    }
}

__global__ void reset_counter_kernel(unsigned long long* c)
{
    if (threadIdx.x < ORBG_XCDS) c[threadIdx.x * ORBG_COUNTER_STRIDE] = 0ull;
}

template <int NK, bool ORDERED, typename S>
static void launch_one(const DecodeArgs& a, int64_t wgs, int chunk, hipStream_t stream)
{
    decode_kernel<NK, ORDERED, S><<<(unsigned)wgs, ORBG_WAVE, 0, stream>>>(
        a.llr, a.nblocks, a.n, a.cols, a.sched, a.bh, (uint32_t)a.slen, a.rdepth, (uint32_t)a.budget,
        a.order, a.cw, a.queries, a.abandoned, a.work, chunk);
}

template <int NK>
static hipError_t launch_nk(const DecodeArgs& a, hipStream_t stream)
{
    int64_t wgs = a.nblocks;
    if (a.max_workgroups > 0 && wgs > a.max_workgroups) wgs = a.max_workgroups;
    if (wgs < 1) return hipSuccess;
    // about 16 chunks per wave: few atomics, and a short tail when blocks differ
    int chunk = a.chunk;
    if (chunk <= 0) {
        const int64_t c = a.nblocks / (wgs * 16);
        chunk = (int)(c < 1 ? 1 : (c > 64 ? 64 : c));
    }
    reset_counter_kernel<<<1, 64, 0, stream>>>(a.work);
    const bool s32 = a.m <= 32;
    if (a.order) {
        if (s32) launch_one<NK, true, uint32_t>(a, wgs, chunk, stream);
        else launch_one<NK, true, uint64_t>(a, wgs, chunk, stream);
    } else {
        if (s32) launch_one<NK, false, uint32_t>(a, wgs, chunk, stream);
        else launch_one<NK, false, uint64_t>(a, wgs, chunk, stream);
    }
    return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs& a, hipStream_t stream)
{
    const int nk = (a.n + ORBG_WAVE - 1) / ORBG_WAVE;
    if (nk <= 1) return launch_nk<1>(a, stream);
    if (nk <= 2) return launch_nk<2>(a, stream);
    if (nk <= 4) return launch_nk<4>(a, stream);
    if (nk <= 8) return launch_nk<8>(a, stream);
    return launch_nk<16>(a, stream);
}

}  // namespace orbg
