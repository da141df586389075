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
//      register bitonic network (stable by index, Sec. III-A permutation);
//      the columns of the R least reliable bits are written to LDS in rank order
//      (h_j = column of the j-th least reliable bit, h_0 = 0);
//   4. search: the wave tests 64 consecutive schedule entries per step, lane l
//      taking entry 64t + l; its syndrome is s0 XOR h_{v_1} XOR ... XOR h_{v_w}
//      (linearity of the parity-check product, Sec. I), a ballot of
//      "syndrome == 0" gives the lowest-index hit, so the result is the first
//      code-book member in schedule order whatever the lane timing;
//   5. output: codeword in received order, queries used, abandon flag (the
//      budget is exhausted without a hit, Sec. IV-A).
//
// With a batch order (learned proposal) step t < 64 tests batch order[t] of the
// schedule instead of batch t; from step 64 on the plain order continues.
#include "orbg_device.h"
#include "orbg_internal.h"
#include "orbg_kernels.h"

namespace orbg {

template <int NK>
__device__ __forceinline__ void decode_block(
    const float* __restrict__ llr_row, int n, const uint64_t* __restrict__ s_cols,
    uint64_t* __restrict__ s_h, uint16_t* __restrict__ s_pi,
    const uint4* __restrict__ sched, const uint8_t* __restrict__ bw, uint64_t slen, int rdepth,
    uint64_t budget, const uint8_t* __restrict__ order_row,
    uint8_t* __restrict__ cw_row, uint64_t* __restrict__ q_out, uint8_t* __restrict__ ab_out)
{
    const int lane = lane_id();

    // 1-2. stage, hard decision, base syndrome
    float x[NK];
    uint64_t acc = 0;
    bool ybit[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane;
        x[j] = (i < n) ? llr_row[i] : 0.0f;
        ybit[j] = (i < n) && (x[j] > 0.0f);
        acc ^= ybit[j] ? s_cols[i] : 0ull;
    }
    const uint64_t s0 = wave_xor_reduce(acc);

    bool found = false;
    uint64_t q = budget;
    uint4 win = make_uint4(0u, 0u, 0u, 0u);

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
        if (lane == 0) { s_h[0] = 0ull; s_pi[0] = 0; }
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int e = lane * NK + j;          // rank e + 1
            if (e < rdepth) {
                const uint32_t idx = (uint32_t)key[j];
                s_h[e + 1] = s_cols[idx];
                s_pi[e + 1] = (uint16_t)idx;
            }
        }
        wave_lds_sync();

        // 4. search
        for (uint64_t t = 0;; ++t) {
            const uint64_t first_pos = t * ORBG_WAVE;            // queries before this step
            if (first_pos >= budget) break;
            uint64_t batch = t;
            if (order_row != nullptr && t < 64) batch = order_row[t];
            const uint64_t g = batch * ORBG_WAVE + lane;
            const bool valid = (first_pos + lane < budget) && (g < slen);
            const uint4 ent = valid ? sched[g] : make_uint4(0u, 0u, 0u, 0u);
            const int wb = (batch * ORBG_WAVE < slen) ? bw[batch] : 0;
            const uint32_t word[4] = {ent.x, ent.y, ent.z, ent.w};
            uint64_t s = s0;
#pragma unroll
            for (int u = 0; u < ORBG_ENTRY_RANKS; ++u) {
                if (u < wb) {
                    const uint32_t r = (word[u >> 2] >> (8 * (u & 3))) & 0xffu;
                    s ^= s_h[r];
                }
            }
            const uint64_t hits = ballot(valid && s == 0);
            if (hits) {
                const int wl = __builtin_ctzll(hits);
                found = true;
                q = first_pos + wl + 1;
                win.x = __shfl(ent.x, wl, ORBG_WAVE);
                win.y = __shfl(ent.y, wl, ORBG_WAVE);
                win.z = __shfl(ent.z, wl, ORBG_WAVE);
                win.w = __shfl(ent.w, wl, ORBG_WAVE);
                break;
            }
            if (order_row == nullptr && (t + 1) * ORBG_WAVE >= slen) break;
            if (order_row != nullptr && t >= 64 && (t + 1) * ORBG_WAVE >= slen) break;
        }
    }

    // 5. output: flip the winning pattern's positions
    const uint32_t wword[4] = {win.x, win.y, win.z, win.w};
    int flip_pos[ORBG_ENTRY_RANKS];
#pragma unroll
    for (int u = 0; u < ORBG_ENTRY_RANKS; ++u) {
        const uint32_t r = (wword[u >> 2] >> (8 * (u & 3))) & 0xffu;
        flip_pos[u] = (found && r != 0) ? (int)s_pi[r] : -1;
    }
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane;
        if (i < n) {
            bool b = ybit[j];
#pragma unroll
            for (int u = 0; u < ORBG_ENTRY_RANKS; ++u) b ^= (flip_pos[u] == i);
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
              const uint4* __restrict__ sched, const uint8_t* __restrict__ bw, uint64_t slen, int rdepth,
              uint64_t budget, const uint8_t* __restrict__ order,
              uint8_t* __restrict__ cw, uint64_t* __restrict__ queries, uint8_t* __restrict__ abandoned)
{
    __shared__ uint64_t s_cols[ORBG_WAVE * NK];
    __shared__ uint64_t s_h[WAVES][ORBG_RANK_SLOTS];
    __shared__ uint16_t s_pi[WAVES][ORBG_RANK_SLOTS];
    for (int i = threadIdx.x; i < n; i += WAVES * ORBG_WAVE) s_cols[i] = cols[i];
    __syncthreads();
    const int wave = threadIdx.x / ORBG_WAVE;
    const int64_t stride = (int64_t)gridDim.x * WAVES;
    for (int64_t b = (int64_t)blockIdx.x * WAVES + wave; b < nblocks; b += stride) {
        decode_block<NK>(llr + b * n, n, s_cols, s_h[wave], s_pi[wave], sched, bw, slen, rdepth, budget,
                         order ? order + b * 64 : nullptr, cw + b * n, queries + b, abandoned + b);
    }
}

template <int NK>
static hipError_t launch_nk(const DecodeArgs& a, hipStream_t stream)
{
    constexpr int WAVES = 4;
    int64_t wgs = (a.nblocks + WAVES - 1) / WAVES;
    if (a.max_workgroups > 0 && wgs > a.max_workgroups) wgs = a.max_workgroups;
    if (wgs < 1) return hipSuccess;
    decode_kernel<NK, WAVES><<<(unsigned)wgs, WAVES * ORBG_WAVE, 0, stream>>>(
        a.llr, a.nblocks, a.n, a.cols, a.sched, a.bw, a.slen, a.rdepth, a.budget, a.order,
        a.cw, a.queries, a.abandoned);
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
