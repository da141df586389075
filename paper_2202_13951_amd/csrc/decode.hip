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

struct WaveLds {
    uint64_t T[256];                    // s0 ^ syndromes of subsets of ranks 1..8
    uint64_t h[ORBG_RANK_SLOTS];        // h[r] = column of rank r (h[0] = 0)
    uint16_t pi[ORBG_RANK_SLOTS];       // pi[r] = received index of rank r
};

__device__ __forceinline__ uint32_t entry_byte(const uint2 e, int u)
{
    return (u < 4) ? ((e.x >> (8 * u)) & 0xffu) : ((e.y >> (8 * (u - 4))) & 0xffu);
}

template <int NK>
__device__ __forceinline__ void load_row(const float* __restrict__ llr_row, int n, float (&x)[NK])
{
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane_id();
        x[j] = (i < n) ? llr_row[i] : 0.0f;
    }
}

template <int NK>
__device__ __forceinline__ void decode_block(
    const float (&x)[NK], int n, const uint64_t* __restrict__ s_cols, WaveLds& L,
    const uint2* __restrict__ sched, const uint8_t* __restrict__ bh, uint64_t slen, int rdepth,
    uint64_t budget, const uint8_t* __restrict__ order_row,
    uint8_t* __restrict__ cw_row, uint64_t* __restrict__ q_out, uint8_t* __restrict__ ab_out)
{
    const int lane = lane_id();

    // 1-2. hard decision, base syndrome (the row was staged by the caller)
    uint64_t acc = 0;
    bool ybit[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane;
        ybit[j] = (i < n) && (x[j] > 0.0f);
        acc ^= ybit[j] ? s_cols[i] : 0ull;
    }
    const uint64_t s0 = wave_xor_reduce(acc);

    bool found = false;
    uint64_t q = budget;
    uint2 win = make_uint2(0u, 0u);

    if (s0 == 0 && order_row == nullptr) {
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
        if (lane == 0) { L.h[0] = 0ull; L.pi[0] = 0; }
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int e = lane * NK + j;          // rank e + 1
            if (e < rdepth) {
                const uint32_t idx = (uint32_t)key[j];
                L.h[e + 1] = s_cols[idx];
                L.pi[e + 1] = (uint16_t)idx;
            } else if (e < ORBG_LOW_RANKS) {
                L.h[e + 1] = 0ull;                // ranks beyond n (tiny codes)
            }
        }
        wave_lds_sync();
        uint64_t a = s0;
#pragma unroll
        for (int b = 0; b < 6; ++b) a ^= ((lane >> b) & 1) ? L.h[b + 1] : 0ull;
        const uint64_t h7 = L.h[7], h8 = L.h[8];
        L.T[lane] = a;
        L.T[lane + 64] = a ^ h7;
        L.T[lane + 128] = a ^ h8;
        L.T[lane + 192] = a ^ h7 ^ h8;
        wave_lds_sync();

        // 4. search (step t tests batch bt = order[t] or t; lane l takes entry 64 bt + l,
        // which is query number 64 t + l + 1)
        uint64_t t = 0;
        uint64_t bt = (order_row != nullptr) ? (order_row[0] & 63u) : 0;
        uint64_t g = bt * ORBG_WAVE + lane;
        bool valid = ((uint64_t)lane < budget) && (g < slen);
        uint2 ent = valid ? sched[g] : make_uint2(0u, 0u);
        int nh = bh[bt];
        for (;;) {
            const uint64_t t1 = t + 1;
            const uint64_t b1 = (order_row != nullptr && t1 < 64) ? (order_row[t1] & 63u) : t1;
            const bool has_next = (t1 * ORBG_WAVE < budget) && (b1 * ORBG_WAVE < slen);
            uint2 ent1 = make_uint2(0u, 0u);
            int nh1 = 0;
            bool valid1 = false;
            if (has_next) {
                const uint64_t g1 = b1 * ORBG_WAVE + lane;
                valid1 = (t1 * ORBG_WAVE + lane < budget) && (g1 < slen);
                if (valid1) ent1 = sched[g1];
                nh1 = bh[b1];
            }
            uint64_t s = L.T[ent.x & 0xffu];
#pragma unroll
            for (int u = 1; u <= ORBG_HIGH_SLOTS; ++u)
                if (u <= nh) s ^= L.h[entry_byte(ent, u)];
            const uint64_t hits = ballot(valid && s == 0);
            if (hits) {
                const int wl = __builtin_ctzll(hits);
                found = true;
                q = t * ORBG_WAVE + wl + 1;
                win.x = __shfl(ent.x, wl, ORBG_WAVE);
                win.y = __shfl(ent.y, wl, ORBG_WAVE);
                break;
            }
            if (!has_next) break;
            t = t1; ent = ent1; nh = nh1; valid = valid1;
        }
    }

    // 5. output: flip the winning pattern's positions
    int flip_pos[ORBG_LOW_RANKS + ORBG_HIGH_SLOTS];
#pragma unroll
    for (int u = 0; u < ORBG_LOW_RANKS; ++u)
        flip_pos[u] = (found && ((win.x >> u) & 1u)) ? (int)L.pi[u + 1] : -1;
#pragma unroll
    for (int u = 1; u <= ORBG_HIGH_SLOTS; ++u) {
        const uint32_t r = entry_byte(win, u);
        flip_pos[ORBG_LOW_RANKS + u - 1] = (found && r != 0) ? (int)L.pi[r] : -1;
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
    if (lane == 0) {
        *q_out = found ? q : budget;
        *ab_out = found ? 0 : 1;
    }
    wave_lds_sync();
}

template <int NK, int WAVES>
__global__ void __launch_bounds__(WAVES * ORBG_WAVE)
decode_kernel(const float* __restrict__ llr, int64_t nblocks, int n,
              const uint64_t* __restrict__ cols,
              const uint2* __restrict__ sched, const uint8_t* __restrict__ bh, uint64_t slen, int rdepth,
              uint64_t budget, const uint8_t* __restrict__ order,
              uint8_t* __restrict__ cw, uint64_t* __restrict__ queries, uint8_t* __restrict__ abandoned,
              unsigned long long* __restrict__ work, int chunk)
{
    __shared__ uint64_t s_cols[ORBG_WAVE * NK];
    __shared__ WaveLds s_wave[WAVES];
    for (int i = threadIdx.x; i < n; i += WAVES * ORBG_WAVE) s_cols[i] = cols[i];
    __syncthreads();
    const int wave = threadIdx.x / ORBG_WAVE;
    WaveLds& L = s_wave[wave];
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
                decode_block<NK>(x, n, s_cols, L, sched, bh, slen, rdepth, budget,
                                 order ? order + b * 64 : nullptr, cw + b * n, queries + b, abandoned + b);
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

template <int NK>
static hipError_t launch_nk(const DecodeArgs& a, hipStream_t stream)
{
    constexpr int WAVES = 4;
    int64_t wgs = (a.nblocks + WAVES - 1) / WAVES;
    if (a.max_workgroups > 0 && wgs > a.max_workgroups) wgs = a.max_workgroups;
    if (wgs < 1) return hipSuccess;
    // about 16 chunks per wave: few atomics, and a short tail when blocks differ
    int chunk = a.chunk;
    if (chunk <= 0) {
        const int64_t c = a.nblocks / (wgs * WAVES * 16);
        chunk = (int)(c < 1 ? 1 : (c > 64 ? 64 : c));
    }
    reset_counter_kernel<<<1, 64, 0, stream>>>(a.work);
    decode_kernel<NK, WAVES><<<(unsigned)wgs, WAVES * ORBG_WAVE, 0, stream>>>(
        a.llr, a.nblocks, a.n, a.cols, a.sched, a.bh, a.slen, a.rdepth, a.budget, a.order,
        a.cw, a.queries, a.abandoned, a.work, chunk);
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
