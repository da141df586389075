// Basic ORBGRAND decode kernels for gfx950.
//
// Per block (Algorithm 1 with the basic ORBGRAND generator):
//   1. stage: the block's LLR row is read coalesced (lane l holds elements
//      l, l+64, ...); the code's packed parity-check columns sit in LDS;
//   2. hard decision y_i = [LLR_i > 0] (Sec. III-A) and base syndrome
//      s0 = XOR of the columns with y_i = 1; s0 == 0 means query 1 (no flip) is
//      a code-book member and nothing else is needed;
//   3. rank: keys (IEEE bits of |LLR_i|) << 32 | i sorted ascending by a
//      register bitonic network (stable by index, the permutation of Sec. III-A);
//      h_j = column of the j-th least reliable bit is written to LDS for the
//      ranks the schedule can reach, and T[m] = s0 XOR (XOR of h_j over the bits
//      of m) for all 256 subsets m of ranks 1..8;
//   4. search: a wave tests 64 consecutive schedule entries per step, lane l
//      taking entry 64t + l; its syndrome is T[low mask] XOR h_r over the
//      entry's ranks above 8 (the parity-check product is linear, Sec. I), and a
//      ballot of "syndrome == 0" gives the lowest-index hit, so the result is
//      the first code-book member in schedule order whatever the timing;
//   5. output: codeword in received order, queries used, abandon flag (budget
//      exhausted without a hit, Sec. IV-A).
//
// Two passes.  The light pass runs persistent one-wave workgroups over all
// blocks (XCD-aware work counters); it gives up on a block after `split_steps`
// steps and appends it to a heavy list.  The heavy pass runs persistent
// workgroups of G waves, one heavy block per workgroup: wave 0 builds the
// block's tables in shared LDS, the G waves take steps split, split+1, ... in
// turn, and an LDS atomicMin keeps the earliest hit, so the answer is again the
// first member in schedule order, independent of which wave found what when.
// A launch may mix codes: each block names its code and its row offset.
// With a batch order (learned proposal) step t < 64 tests batch order[t] of the
// schedule instead of batch t; from step 64 on the plain order continues.
#include "orbg_device.h"
#include "orbg_internal.h"
#include "orbg_kernels.h"

namespace orbg {

// Per-block LDS tables: the syndrome type S is u32 when n - k <= 32, else u64.
template <typename S>
struct BlockLds {
    S T[256];                           // s0 ^ syndromes of the subsets of ranks 1..8
    S h[ORBG_RANK_SLOTS];               // h[r] = column of rank r (h[0] = 0)
    uint16_t pi[ORBG_RANK_SLOTS];       // pi[r] = received index of rank r
};

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    return (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32)) << 32) |
                     __builtin_amdgcn_readfirstlane((uint32_t)u));
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

// Read-only tables read with wave-uniform indices: through the constant
// address space so that the loads are scalar (s_load) and need no readfirstlane.
typedef const __attribute__((address_space(4))) uint32_t* const_u32_ptr;
__device__ __forceinline__ uint32_t scalar_load(const uint32_t* p, uint32_t i)
{
    return ((const_u32_ptr)p)[i];
}

// Schedule entry `idx` (idx < 2^22): a 32-bit byte offset from the uniform base
// lets the load use the scalar-base addressing mode.
__device__ __forceinline__ uint2 load_entry(const uint2* __restrict__ sched, uint32_t idx)
{
    return *reinterpret_cast<const uint2*>(reinterpret_cast<const unsigned char*>(sched) + (idx << 3));
}

// Mask of the lowest `cnt` lanes.
__device__ __forceinline__ uint64_t low_lanes(uint32_t cnt) { return cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull); }

// A block's batch order held in registers: lane l keeps byte l of its row
// (values taken modulo 64), read once per block.
template <bool ORDERED>
__device__ __forceinline__ uint32_t load_order(const uint8_t* __restrict__ order_row)
{
    return ORDERED ? ((uint32_t)order_row[lane_id()] & 63u) : 0u;
}

// Batch tested at step t: the block's order for the first 64 steps, the plain
// order afterwards.
template <bool ORDERED>
__device__ __forceinline__ uint32_t batch_at(uint32_t ordv, uint32_t t)
{
    if (!ORDERED || t >= 64) return t;
    return (uint32_t)__builtin_amdgcn_readlane((int)ordv, (int)t);
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

// Steps 1-2: hard decision bits and base syndrome (wave-uniform).
template <int NK, typename S>
__device__ __forceinline__ S hard_decision(const float (&x)[NK], int n, const S* __restrict__ cols, bool (&ybit)[NK])
{
    const int lane = lane_id();
    S acc = 0;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane;
        ybit[j] = (i < n) && (x[j] > 0.0f);
        acc ^= ybit[j] ? cols[i] : (S)0;
    }
    return wave_xor_reduce_s<S>(acc);
}

// Step 3: reliability order and the per-block lookup tables.
template <int NK, typename S>
__device__ __forceinline__ void rank_and_tables(const float (&x)[NK], int n, const S* __restrict__ cols, S s0,
                                                int rdepth, BlockLds<S>& L)
{
    const int lane = lane_id();
    uint64_t key[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane;
        key[j] = (i < n) ? (((uint64_t)(__float_as_uint(x[j]) & 0x7fffffffu) << 32) | (uint32_t)i) : ~0ull;
    }
    bitonic_sort<NK>(key);
    wave_lds_sync();
    if (lane == 0) { L.h[0] = 0; L.pi[0] = 0; }
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int e = lane * NK + j;          // rank e + 1
        if (e < rdepth) {
            const uint32_t idx = (uint32_t)key[j];
            L.h[e + 1] = cols[idx];
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
}

// Step 4, one step: syndrome of every lane's entry (all LDS reads before the XORs).
template <typename S>
__device__ __forceinline__ S entry_syndrome(const BlockLds<S>& L, uint2 ent, uint32_t nh)
{
    const S v0 = L.T[ent.x & 0xffu];
    S v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0, v6 = 0, v7 = 0;
    if (nh >= 1) v1 = L.h[(ent.x >> 8) & 0xffu];
    if (nh >= 2) v2 = L.h[(ent.x >> 16) & 0xffu];
    if (nh >= 3) v3 = L.h[ent.x >> 24];
    if (nh >= 4) v4 = L.h[ent.y & 0xffu];
    if (nh >= 5) v5 = L.h[(ent.y >> 8) & 0xffu];
    if (nh >= 6) v6 = L.h[(ent.y >> 16) & 0xffu];
    if (nh >= 7) v7 = L.h[ent.y >> 24];
    return v0 ^ v1 ^ v2 ^ v3 ^ v4 ^ v5 ^ v6 ^ v7;
}

// Step 5: the hard decision with the winning entry's ranks flipped.
template <int NK, typename S>
__device__ __forceinline__ void write_codeword(const bool (&ybit)[NK], int n, const BlockLds<S>& L,
                                               uint32_t win_lo, uint32_t win_hi, uint8_t* __restrict__ cw_row)
{
    const int lane = lane_id();
    if ((win_lo | win_hi) == 0) {
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int i = j * ORBG_WAVE + lane;
            if (i < n) cw_row[i] = ybit[j] ? 1 : 0;
        }
        return;
    }
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

// Light pass, one block.  Returns true if the block is left for the heavy pass
// (then nothing is written).
template <int NK, bool ORDERED, typename S>
__device__ __forceinline__ bool light_block(
    const float (&x)[NK], const CodeDesc& c, const S* __restrict__ cols, BlockLds<S>& L,
    uint32_t budget, uint32_t split_steps, const uint8_t* __restrict__ order_row,
    uint8_t* __restrict__ cw_row, uint64_t* __restrict__ q_out, uint8_t* __restrict__ ab_out)
{
    const int lane = lane_id();
    const int n = c.n;
    bool ybit[NK];
    const uint32_t ordv = load_order<ORDERED>(order_row);
    const S s0 = hard_decision<NK, S>(x, n, cols, ybit);

    bool found = false;
    uint32_t q = budget;
    uint32_t win_lo = 0, win_hi = 0;     // winning entry (wave-uniform)

    // s0 == 0: the empty pattern (entry 0 of batch 0) is a member; it is the first
    // hit when batch 0 is tested first (always in the plain order)
    if (s0 == 0 && (!ORDERED || batch_at<ORDERED>(ordv, 0) == 0)) {
        found = true;
        q = 1;
    } else {
        rank_and_tables<NK, S>(x, n, cols, s0, c.rdepth, L);
        const uint2* __restrict__ sched = c.sched;
        const uint32_t* __restrict__ bh = c.bh;
        const uint32_t slen = c.slen;
        // Step t tests batch bt; lane l takes schedule entry 64 bt + l, which is
        // query number 64 t + l + 1.  Lanes past the budget or the schedule read a
        // valid entry and are masked out of the ballot.  Indices fit 32 bits.
        uint32_t t = 0;
        const uint32_t bt = batch_at<ORDERED>(ordv, 0);
        uint64_t vmA = low_lanes(min(budget, slen - bt * ORBG_WAVE));
        uint2 entA = load_entry(sched, min(bt * ORBG_WAVE + lane, slen - 1));
        uint32_t nhA = scalar_load(bh, bt);
        uint2 entB = make_uint2(0u, 0u);
        uint32_t nhB = 0;
        uint64_t vmB = 0;
        // One step: load the next step's entries, test the current ones.
        // Returns 0 (go on), 1 (hit), 2 (no hit, nothing left), 3 (split point).
        // The loop alternates two register sets, so a load is consumed one full
        // step after it was issued.
        auto step = [&](const uint2 cur, const uint32_t nh_cur, const uint64_t vm_cur, uint2& nxt,
                        uint32_t& nh_nxt, uint64_t& vm_nxt) -> int {
            const uint32_t t1 = t + 1;
            const uint32_t b1 = batch_at<ORDERED>(ordv, t1);
            const bool has_next = (t1 * ORBG_WAVE < budget) && (b1 * ORBG_WAVE < slen);
            // loads issued on every path (a valid batch when there is no next
            // step), so the wait for the current entries never covers them
            const uint32_t bl = has_next ? b1 : 0u;
            nxt = load_entry(sched, min(bl * ORBG_WAVE + lane, slen - 1));
            nh_nxt = scalar_load(bh, bl);
            vm_nxt = has_next ? low_lanes(min(budget - t1 * ORBG_WAVE, slen - b1 * ORBG_WAVE)) : 0ull;
            const S syn = entry_syndrome<S>(L, cur, nh_cur);
            const uint64_t hits = ballot(syn == 0) & vm_cur;
            if (hits) {
                const int wl = __builtin_ctzll(hits);
                q = t * ORBG_WAVE + wl + 1;
                win_lo = __builtin_amdgcn_readlane(cur.x, wl);
                win_hi = __builtin_amdgcn_readlane(cur.y, wl);
                return 1;
            }
            if (!has_next) return 2;
            if (split_steps != 0 && t1 >= split_steps) return 3;
            t = t1;
            return 0;
        };
        int r;
        for (;;) {
            if ((r = step(entA, nhA, vmA, entB, nhB, vmB)) != 0) break;
            if ((r = step(entB, nhB, vmB, entA, nhA, vmA)) != 0) break;
        }
        if (r == 3) {
            wave_lds_sync();
            return true;
        }
        found = (r == 1);
    }

    write_codeword<NK, S>(ybit, n, L, win_lo, win_hi, cw_row);
    if (lane == 0) {
        *q_out = found ? q : budget;
        *ab_out = found ? 0 : 1;
    }
    wave_lds_sync();
    return false;
}

template <int NK, bool ORDERED, typename S>
__device__ __forceinline__ void light_one(const float (&x)[NK], const CodeDesc& c, const S* cols, BlockLds<S>& L,
                                          int64_t b, int64_t row, uint32_t budget, uint32_t split_steps,
                                          const uint8_t* order, uint8_t* cw, uint64_t* queries,
                                          uint8_t* abandoned, unsigned long long* ctrs, int64_t* heavy)
{
    const bool left = light_block<NK, ORDERED, S>(x, c, cols, L, budget, split_steps,
                                                  ORDERED ? order + b * 64 : nullptr, cw + row, queries + b,
                                                  abandoned + b);
    if (left && lane_id() == 0) {
        const unsigned long long slot = atomicAdd(ctrs + ORBG_CTR_HEAVY_COUNT, 1ull);
        heavy[slot] = b;
    }
}

// Light pass.  One wave per workgroup, so the wave's LDS tables sit at fixed
// addresses.  MIXED: each block names its code (block_code) and row offset;
// otherwise all blocks use code 0 with rows b * n.  NKMAX: largest keys per
// lane among the launch's codes.
template <int NKMAX, bool ORDERED, typename S, bool MIXED>
__global__ void __launch_bounds__(ORBG_WAVE)
light_kernel(CodeTable codes, const uint8_t* __restrict__ block_code, const int64_t* __restrict__ row_off,
             const float* __restrict__ llr, int64_t nblocks, uint32_t budget, uint32_t split_steps,
             const uint8_t* __restrict__ order, uint8_t* __restrict__ cw, uint64_t* __restrict__ queries,
             uint8_t* __restrict__ abandoned, unsigned long long* __restrict__ ctrs, int64_t* __restrict__ heavy,
             int chunk)
{
    // columns of the launch's codes: sum of n entries (dynamic LDS, sized at launch)
    extern __shared__ __align__(16) unsigned char orbg_dyn_lds[];
    S* s_cols = reinterpret_cast<S*>(orbg_dyn_lds);
    __shared__ BlockLds<S> L;
    for (int ci = 0; ci < (MIXED ? codes.ncodes : 1); ++ci)
        for (int i = threadIdx.x; i < codes.c[ci].n; i += ORBG_WAVE)
            s_cols[codes.c[ci].col_base + i] = (S)codes.c[ci].cols[i];
    wave_lds_sync();
    const int lane = lane_id();

    // XCD-aware work split: workgroups are dealt round-robin to the 8 XCDs, so
    // workgroup w works first on slice w % 8 of the blocks through that slice's
    // counter (an atomic in the XCD's own L2), then helps the other slices.
    const int home = (int)(blockIdx.x % ORBG_XCDS);
    for (int k = 0; k < ORBG_XCDS; ++k) {
        const int xs = (home + k) % ORBG_XCDS;
        const int64_t lo = nblocks * xs / ORBG_XCDS, hi = nblocks * (xs + 1) / ORBG_XCDS;
        unsigned long long* ctr = ctrs + ORBG_CTR_SLICE(xs);
        unsigned long long c0 = 0;
        if (lane == 0) c0 = atomicAdd(ctr, (unsigned long long)chunk);
        int64_t b0 = lo + (int64_t)__shfl(c0, 0, ORBG_WAVE);
        while (b0 < hi) {
            unsigned long long c1 = 0;
            if (lane == 0) c1 = atomicAdd(ctr, (unsigned long long)chunk);   // in flight meanwhile
            const int64_t end = (b0 + chunk < hi) ? b0 + chunk : hi;
            if (!MIXED) {
                constexpr int NK = NKMAX;
                const CodeDesc& c = codes.c[0];
                float x[NK];
                load_row<NK>(llr + b0 * c.n, c.n, x);
                for (int64_t b = b0; b < end; ++b) {
                    float xn[NK];
                    if (b + 1 < end) load_row<NK>(llr + (b + 1) * c.n, c.n, xn);   // next row in flight
                    light_one<NK, ORDERED, S>(x, c, s_cols, L, b, b * c.n, budget, split_steps, order, cw,
                                              queries, abandoned, ctrs, heavy);
#pragma unroll
                    for (int j = 0; j < NK; ++j) x[j] = xn[j];
                }
            } else {
                for (int64_t b = b0; b < end; ++b) {
                    int ci = (int)uniform_u32(block_code[b]);
                    ci = ci < codes.ncodes ? ci : 0;      // out-of-range indices read code 0
                    const CodeDesc& c = codes.c[ci];
                    const int64_t row = uniform_i64(row_off[b]);
                    const S* cols = s_cols + c.col_base;
                    if (c.nk == 1 || NKMAX == 1) {
                        float x[1];
                        load_row<1>(llr + row, c.n, x);
                        light_one<1, ORDERED, S>(x, c, cols, L, b, row, budget, split_steps, order, cw, queries,
                                                 abandoned, ctrs, heavy);
                    } else if (c.nk == 2 || NKMAX == 2) {
                        constexpr int K2 = NKMAX >= 2 ? 2 : 1;
                        float x[K2];
                        load_row<K2>(llr + row, c.n, x);
                        light_one<K2, ORDERED, S>(x, c, cols, L, b, row, budget, split_steps, order, cw, queries,
                                                  abandoned, ctrs, heavy);
                    } else {
                        float x[NKMAX];
                        load_row<NKMAX>(llr + row, c.n, x);
                        light_one<NKMAX, ORDERED, S>(x, c, cols, L, b, row, budget, split_steps, order, cw,
                                                     queries, abandoned, ctrs, heavy);
                    }
                }
            }
            b0 = lo + (int64_t)__shfl(c1, 0, ORBG_WAVE);
        }
    }
}

// Heavy pass, one block shared by the workgroup's G waves (all waves call it).
// Plain order only: blocks reach it after at least 64 steps or were never reordered.
template <int NK, typename S, int G>
__device__ __forceinline__ void heavy_block(const CodeDesc& c, const float* __restrict__ llr_row, S* s_cols,
                                            BlockLds<S>& L, uint32_t* best, uint32_t budget, uint32_t split_steps,
                                            uint8_t* __restrict__ cw_row, uint64_t* __restrict__ q_out,
                                            uint8_t* __restrict__ ab_out)
{
    const int lane = lane_id();
    const int wave = threadIdx.x / ORBG_WAVE;
    const int n = c.n;
    for (int i = threadIdx.x; i < n; i += G * ORBG_WAVE) s_cols[i] = (S)c.cols[i];
    if (threadIdx.x == 0) *best = 0xffffffffu;
    __syncthreads();
    float x[NK];
    bool ybit[NK];
    if (wave == 0) {
        load_row<NK>(llr_row, n, x);
        const S s0 = hard_decision<NK, S>(x, n, s_cols, ybit);
        rank_and_tables<NK, S>(x, n, s_cols, s0, c.rdepth, L);
    }
    __syncthreads();
    const uint2* __restrict__ sched = c.sched;
    const uint32_t slen = c.slen;
    // wave w takes steps split + w, split + w + G, ...; the next one's entries
    // are loaded while the current one is tested
    uint32_t t = split_steps + wave;
    if (t * ORBG_WAVE < budget && t * ORBG_WAVE < slen) {
        uint2 entA = load_entry(sched, min(t * ORBG_WAVE + lane, slen - 1));
        uint32_t nhA = scalar_load(c.bh, t);
        uint2 entB = make_uint2(0u, 0u);
        uint32_t nhB = 0;
        // returns true when this wave is done (hit, nothing left, or an earlier hit known)
        auto step = [&](const uint2 cur, const uint32_t nh_cur, uint2& nxt, uint32_t& nh_nxt) -> bool {
            if (t * ORBG_WAVE + 1 > __hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                return true;
            const uint32_t t1 = t + G;
            const bool has_next = t1 * ORBG_WAVE < budget && t1 * ORBG_WAVE < slen;
            const uint32_t tl = has_next ? t1 : t;            // loads on every path
            nxt = load_entry(sched, min(tl * ORBG_WAVE + lane, slen - 1));
            nh_nxt = scalar_load(c.bh, tl);
            const uint64_t vmask = low_lanes(min(budget - t * ORBG_WAVE, slen - t * ORBG_WAVE));
            const S syn = entry_syndrome<S>(L, cur, nh_cur);
            const uint64_t hits = ballot(syn == 0) & vmask;
            if (hits) {
                if (lane == 0) atomicMin(best, t * ORBG_WAVE + (uint32_t)__builtin_ctzll(hits) + 1);
                return true;
            }
            if (!has_next) return true;
            t = t1;
            return false;
        };
        for (;;) {
            if (step(entA, nhA, entB, nhB)) break;
            if (step(entB, nhB, entA, nhA)) break;
        }
    }
    __syncthreads();
    if (wave == 0) {
        const uint32_t q = uniform_u32(*best);
        const bool found = q != 0xffffffffu;
        uint32_t win_lo = 0, win_hi = 0;
        if (found) {
            const uint2 w = sched[q - 1];           // plain order: entry index = query number - 1
            win_lo = uniform_u32(w.x);
            win_hi = uniform_u32(w.y);
        }
        write_codeword<NK, S>(ybit, n, L, win_lo, win_hi, cw_row);
        if (lane == 0) {
            *q_out = found ? q : budget;
            *ab_out = found ? 0 : 1;
        }
    }
    __syncthreads();
}

template <int NKMAX, typename S, bool MIXED, int G>
__global__ void __launch_bounds__(G * ORBG_WAVE)
heavy_kernel(CodeTable codes, const uint8_t* __restrict__ block_code, const int64_t* __restrict__ row_off,
             const float* __restrict__ llr, uint32_t budget, uint32_t split_steps,
             uint8_t* __restrict__ cw, uint64_t* __restrict__ queries, uint8_t* __restrict__ abandoned,
             unsigned long long* __restrict__ ctrs, const int64_t* __restrict__ heavy)
{
    __shared__ S s_cols[ORBG_WAVE * NKMAX];
    __shared__ BlockLds<S> L;
    __shared__ uint32_t best;
    __shared__ int64_t cur;
    const unsigned long long count = *(volatile unsigned long long*)(ctrs + ORBG_CTR_HEAVY_COUNT);
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned long long i = atomicAdd(ctrs + ORBG_CTR_HEAVY_NEXT, 1ull);
            cur = (i < count) ? heavy[i] : -1;
        }
        __syncthreads();
        const int64_t b = uniform_i64(cur);
        __syncthreads();
        if (b < 0) break;
        int ci = MIXED ? (int)uniform_u32(block_code[b]) : 0;
        ci = ci < codes.ncodes ? ci : 0;
        const CodeDesc& c = codes.c[ci];
        const int64_t row = MIXED ? uniform_i64(row_off[b]) : b * c.n;
        if (c.nk == 1 || NKMAX == 1) {
            heavy_block<1, S, G>(c, llr + row, s_cols, L, &best, budget, split_steps, cw + row, queries + b,
                                 abandoned + b);
        } else if (c.nk == 2 || NKMAX == 2) {
            constexpr int K2 = NKMAX >= 2 ? 2 : 1;
            heavy_block<K2, S, G>(c, llr + row, s_cols, L, &best, budget, split_steps, cw + row, queries + b,
                                  abandoned + b);
        } else if (c.nk == 4 || NKMAX == 4) {
            constexpr int K4 = NKMAX >= 4 ? 4 : 1;
            heavy_block<K4, S, G>(c, llr + row, s_cols, L, &best, budget, split_steps, cw + row, queries + b,
                                  abandoned + b);
        } else {
            heavy_block<NKMAX, S, G>(c, llr + row, s_cols, L, &best, budget, split_steps, cw + row, queries + b,
                                     abandoned + b);
        }
    }
}

__global__ void reset_counters_kernel(unsigned long long* c)
{
    for (int i = threadIdx.x; i < ORBG_CTR_WORDS; i += blockDim.x) c[i] = 0ull;
}

template <int NKMAX, bool ORDERED, typename S, bool MIXED>
static void launch_light(const DecodeArgs& a, int64_t wgs, int chunk, uint32_t split, hipStream_t stream)
{
    uint32_t ncols = 0;
    for (int i = 0; i < (MIXED ? a.codes.ncodes : 1); ++i) {
        const uint32_t e = a.codes.c[i].col_base + (uint32_t)a.codes.c[i].n;
        ncols = e > ncols ? e : ncols;
    }
    light_kernel<NKMAX, ORDERED, S, MIXED><<<(unsigned)wgs, ORBG_WAVE, ncols * sizeof(S), stream>>>(
        a.codes, a.block_code, a.row_off, a.llr, a.nblocks, a.budget, split, a.order, a.cw, a.queries,
        a.abandoned, a.ctrs, a.heavy, chunk);
}

template <int NKMAX, typename S, bool MIXED, int G>
static void launch_heavy_g(const DecodeArgs& a, uint32_t split, hipStream_t stream)
{
    const int64_t wgs = (int64_t)a.cus * (a.p.heavy_wg_per_cu > 0 ? a.p.heavy_wg_per_cu : 2);
    heavy_kernel<NKMAX, S, MIXED, G><<<(unsigned)wgs, G * ORBG_WAVE, 0, stream>>>(
        a.codes, a.block_code, a.row_off, a.llr, a.budget, split, a.cw, a.queries, a.abandoned, a.ctrs, a.heavy);
}

template <int NKMAX, bool ORDERED, typename S, bool MIXED>
static hipError_t launch_all(const DecodeArgs& a, hipStream_t stream)
{
    int64_t wgs = a.nblocks;
    const int64_t cap = (int64_t)a.cus * (a.p.wg_per_cu > 0 ? a.p.wg_per_cu : 32);
    if (wgs > cap) wgs = cap;
    int chunk = a.p.chunk;
    if (chunk <= 0) {
        const int64_t c = a.nblocks / (wgs * 16);       // about 16 chunks per wave
        chunk = (int)(c < 1 ? 1 : (c > 64 ? 64 : c));
    }
    const uint32_t split = (a.heavy != nullptr && a.p.split_steps > 0) ? (uint32_t)a.p.split_steps : 0u;
    reset_counters_kernel<<<1, 64, 0, stream>>>(a.ctrs);
    launch_light<NKMAX, ORDERED, S, MIXED>(a, wgs, chunk, split, stream);
    if (split) {
        if (a.p.heavy_waves >= 16) launch_heavy_g<NKMAX, S, MIXED, 16>(a, split, stream);
        else if (a.p.heavy_waves >= 8) launch_heavy_g<NKMAX, S, MIXED, 8>(a, split, stream);
        else launch_heavy_g<NKMAX, S, MIXED, 4>(a, split, stream);
    }
    return hipGetLastError();
}

template <int NKMAX, bool MIXED>
static hipError_t launch_nk(const DecodeArgs& a, bool s32, hipStream_t stream)
{
    if (a.order) {
        if (s32) return launch_all<NKMAX, true, uint32_t, MIXED>(a, stream);
        return launch_all<NKMAX, true, uint64_t, MIXED>(a, stream);
    }
    if (s32) return launch_all<NKMAX, false, uint32_t, MIXED>(a, stream);
    return launch_all<NKMAX, false, uint64_t, MIXED>(a, stream);
}

hipError_t launch_decode(const DecodeArgs& a, hipStream_t stream)
{
    if (a.nblocks < 1) return hipSuccess;
    int nk = 1, mmax = 0;
    for (int i = 0; i < a.codes.ncodes; ++i) {
        nk = a.codes.c[i].nk > nk ? a.codes.c[i].nk : nk;
        mmax = a.codes.c[i].m > mmax ? a.codes.c[i].m : mmax;
    }
    const bool s32 = mmax <= 32;
    if (a.mixed) {
        if (nk <= 1) return launch_nk<1, true>(a, s32, stream);
        if (nk <= 2) return launch_nk<2, true>(a, s32, stream);
        if (nk <= 4) return launch_nk<4, true>(a, s32, stream);
        return hipErrorInvalidValue;                    // mixed launches take n <= 256
    }
    if (nk <= 1) return launch_nk<1, false>(a, s32, stream);
    if (nk <= 2) return launch_nk<2, false>(a, s32, stream);
    if (nk <= 4) return launch_nk<4, false>(a, s32, stream);
    if (nk <= 8) return launch_nk<8, false>(a, s32, stream);
    return launch_nk<16, false>(a, s32, stream);
}

}  // namespace orbg
