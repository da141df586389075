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
#pragma once
#include <type_traits>

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

// (readfirstlane returns a signed int: each half is taken as uint32_t before
// widening, or the low half would sign-extend into the high one)
__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
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

// Raw buffer descriptors (gfx9-family word 3: 32-bit data format).  A lane whose
// byte offset lies past `bytes` reads 0 and its store is dropped by the
// hardware, so rows of any length are read and written without branching on the
// lane, which keeps the count of memory operations in flight the same on every
// path and lets the next row's loads and this block's stores stay in flight.
#define ORBG_BUF_DW3 0x00020000
typedef __amdgpu_buffer_rsrc_t buf_t;
typedef uint32_t u32x2_t __attribute__((vector_size(8)));

__device__ __forceinline__ buf_t make_buf(const void* base, uint32_t bytes)
{
    // descriptors live in scalar registers: base and size are wave-uniform
    const uint64_t ua = (uint64_t)uniform_i64((int64_t)(uintptr_t)base);
    return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)ua, 0, (int)__builtin_amdgcn_readfirstlane(bytes),
                                             ORBG_BUF_DW3);
}

template <int NK>
__device__ __forceinline__ void load_row_buf(buf_t r, float (&x)[NK])
{
#pragma unroll
    for (int j = 0; j < NK; ++j)
        x[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (j * ORBG_WAVE + lane_id()) * 4, 0, 0));
}

// Lane offsets of a kernel's row and result accesses, made once per kernel so
// that every access shares the same registers.  l[j] / c[j]: byte offset of
// element j * 64 + lane in an LLR row / a codeword row, or ORBG_PAST for a
// lane past the code's length (one code per launch) — an offset beyond every
// descriptor's size, so the lane reads 0 and its store is dropped;  r: 0 on
// lane 0 and ORBG_PAST elsewhere (a block's query count and flag).
#define ORBG_PAST 0x40000000u
template <int NK>
struct LaneOffs {
    uint32_t l[NK];
    uint32_t c[NK];
    uint32_t r;
};

// n_mask: the length past which lanes are cut (any value >= 64 NK cuts none).
template <int NK>
__device__ __forceinline__ LaneOffs<NK> lane_offsets(int n_mask)
{
    LaneOffs<NK> o;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const uint32_t i = (uint32_t)(j * ORBG_WAVE + lane_id());
        const bool in = i < (uint32_t)n_mask;
        o.l[j] = in ? i * 4u : ORBG_PAST;
        o.c[j] = in ? i : ORBG_PAST;
    }
    o.r = lane_id() == 0 ? 0u : ORBG_PAST;
    return o;
}

// Kernels without a kernel-wide set compute lane offsets in place from the lane
// (none cut).
struct NoOffs {};
template <class LO>
constexpr bool has_offs() { return !std::is_same<LO, NoOffs>::value; }

// A row at byte offset `soff` from the descriptor's base, read with the
// kernel's lane offsets.
template <int NK, class LO>
__device__ __forceinline__ void load_row_buf(buf_t r, float (&x)[NK], const LO& lo, uint32_t soff = 0)
{
    if constexpr (!has_offs<LO>()) {
        load_row_buf<NK>(r, x);
    } else {
#pragma unroll
        for (int j = 0; j < NK; ++j) x[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, lo.l[j], soff, 0));
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
__device__ __forceinline__ uint32_t load_order_buf(buf_t r)
{
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, lane_id(), 0, 0) & 63u;
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

// Rows of H for this lane: lane r < m holds row r as NK words (bit l of word j
// = H[r][64 j + l]), other lanes hold zeros.
template <int NK>
__device__ __forceinline__ void load_hrows(const uint64_t* rows, int m, uint64_t (&h)[NK])
{
    const int r = lane_id() < m ? lane_id() : 0;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const uint64_t w = rows[r * NK + j];
        h[j] = lane_id() < m ? w : 0ull;
    }
}

// Steps 1-2: hard decision bits and base syndrome s0 = H y (wave-uniform).  The
// ballots of y_i = [LLR_i > 0] are the received word as 64-bit words; bit r of
// s0 is the parity of (row r of H) AND y, one row per lane.
template <int NK, typename S>
__device__ __forceinline__ S hard_decision(const float (&x)[NK], int n, const uint64_t (&hrow)[NK],
                                           bool (&ybit)[NK])
{
    const int lane = lane_id();
    // the parity of a sum of popcounts is the parity of the XOR of the words:
    // the masked words are folded first (a AND b XOR c in one three-input bit
    // operation, truth table 0x6a), one popcount at the end
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        ybit[j] = (j * ORBG_WAVE + lane < n) && (x[j] > 0.0f);
        const uint64_t y = ballot(ybit[j]);
        acc = __builtin_amdgcn_bitop3_b32((uint32_t)hrow[j], (uint32_t)y, acc, 0x6a);
        acc = __builtin_amdgcn_bitop3_b32((uint32_t)(hrow[j] >> 32), (uint32_t)(y >> 32), acc, 0x6a);
    }
    return (S)ballot((__popc(acc) & 1u) != 0u);
}

template <int NK>
struct IndexBits { static constexpr int value = NK == 1 ? 6 : NK == 2 ? 7 : NK == 4 ? 8 : NK == 8 ? 9 : 10; };

// Step 3a: received index of every rank, idx[j] for rank lane * NK + j + 1.
// The sort runs on 32-bit keys (top bits of |LLR| above the index); that order
// is the order of the full keys (bits of |LLR|) << 32 | index except inside runs
// of equal truncated magnitudes, so if two neighbours among the ranks the
// schedule reaches share a truncated magnitude, the full 64-bit keys are
// sorted instead; hfit > 0 adds ranks 1 and hfit to the ranks whose element
// must be exact (their magnitudes fit the 1-line model).  Positions past n hold
// keys above every element.
template <int NK>
__device__ __forceinline__ void rank_order(const float (&x)[NK], int n, int rdepth, int hfit, uint32_t (&idx)[NK])
{
    constexpr int IB = IndexBits<NK>::value;
    const int lane = lane_id();
    uint32_t key[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane;
        const uint32_t mag = (i < n) ? (__float_as_uint(x[j]) & 0x7fffffffu) : 0x7fffffffu;
        key[j] = ((mag >> (IB - 1)) << IB) | (uint32_t)i;
    }
    bitonic_sort32<NK>(key);
    const uint32_t next0 = (uint32_t)__shfl_down((int)key[0], 1, ORBG_WAVE);
    bool tie = false;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int e = lane * NK + j;
        const uint32_t other = (j + 1 < NK) ? key[(j + 1) % NK] : next0;
        const bool has_next = (j + 1 < NK) || lane + 1 < ORBG_WAVE;
        const bool exact = e < rdepth || (hfit > 0 && (e == 0 || e == hfit - 2 || e == hfit - 1));
        tie |= has_next && exact && ((key[j] ^ other) >> IB) == 0u;
    }
    if (ballot(tie) != 0ull) {
        uint64_t k64[NK];
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int i = j * ORBG_WAVE + lane;
            k64[j] = (i < n) ? (((uint64_t)(__float_as_uint(x[j]) & 0x7fffffffu) << 32) | (uint32_t)i) : ~0ull;
        }
        bitonic_sort<NK>(k64);
#pragma unroll
        for (int j = 0; j < NK; ++j) idx[j] = (uint32_t)k64[j];
    } else {
#pragma unroll
        for (int j = 0; j < NK; ++j) idx[j] = key[j] & ((1u << IB) - 1u);
    }
}

template <typename S>
__device__ __forceinline__ S readlane_s(S v, int l);
template <>
__device__ __forceinline__ uint32_t readlane_s<uint32_t>(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
template <>
__device__ __forceinline__ uint64_t readlane_s<uint64_t>(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// x of received index i (wave-uniform), read from the lane that holds it.
template <int NK>
__device__ __forceinline__ float value_at(const float (&x)[NK], uint32_t i)
{
    const uint32_t j = i / ORBG_WAVE;
    float v = x[0];
#pragma unroll
    for (int jj = 1; jj < NK; ++jj) v = (j == (uint32_t)jj) ? x[jj] : v;
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)(i % ORBG_WAVE)));
}

// 1-line fit of the sorted reliabilities (Sec. III-E, eqs. (Q) and (quant) with
// one segment and beta = 1): anchors at ranks 1 and h = floor(n / 2), slope
// Q = (L_h - L_1) / (h - 1), offset J0 = [L_1 / Q] - 1 with [x] = floor(x + 1/2),
// each operation rounded to nearest in FP32 in that order.  A slope that is not
// positive and finite, or an L_1 / Q that is not finite, gives J0 = 0 (the
// basic order); [L_1 / Q] is capped at 2^20.  idx[j] holds the received index
// of rank lane * NK + j + 1 (exact for ranks 1 and h).  Returns a wave-uniform
// value.
template <int NK>
__device__ __forceinline__ int fit_offset(const float (&x)[NK], const uint32_t (&idx)[NK], int n)
{
    const int h = n / 2;
    if (h < 2) return 0;
    const uint32_t i1 = (uint32_t)__builtin_amdgcn_readlane((int)idx[0], 0);
    const int e = h - 1;                                  // rank h sits in lane e / NK, key e % NK
    uint32_t sel = idx[0];
#pragma unroll
    for (int j = 1; j < NK; ++j) sel = (e % NK == j) ? idx[j] : sel;
    const uint32_t ih = (uint32_t)__builtin_amdgcn_readlane((int)sel, e / NK);
    const float l1 = fabsf(value_at<NK>(x, i1));
    const float lh = fabsf(value_at<NK>(x, ih));
    const float q = __fdiv_rn(__fsub_rn(lh, l1), (float)(h - 1));
    if (!(q > 0.0f) || !__builtin_isfinite(q)) return 0;
    float r = __fdiv_rn(l1, q);
    if (!__builtin_isfinite(r)) return 0;
    r = floorf(__fadd_rn(r, 0.5f));
    r = r > 1048576.0f ? 1048576.0f : r;
    return (int)uniform_u32((uint32_t)((int)r - 1));
}

// Step 3 for the first batch only: the ra (<= 32) least reliable ranks without
// ranking the whole block.  The threshold t is on the truncated magnitude (the
// key without its index bits), so keys with equal truncated magnitudes fall on
// the same side of it; it moves from the caller's guess (kept from block to
// block) until ra <= #(keys below t) <= 32, at most 8 tries.  The keys below t
// are gathered into lanes 0..31 through LDS and sorted there; lane l < ra then
// holds the received index of rank l + 1.  Returns false when no such t is found
// or when two neighbours among the first ra + 1 gathered keys share a truncated
// magnitude (their order would need the full keys): the caller then ranks the
// whole block.
template <int NK, typename S>
__device__ __forceinline__ bool rank_first(const float (&x)[NK], int n, int ra, uint32_t& guess, BlockLds<S>& L,
                                           uint32_t& idx1)
{
    constexpr int IB = IndexBits<NK>::value;
    constexpr uint32_t PMAX = 1u << (32 - IB);          // truncated magnitudes are < PMAX
    constexpr uint32_t OCT = 1u << (24 - IB);           // one binade in truncated-magnitude units
    const int lane = lane_id();
    uint32_t key[NK];
    bool real[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = j * ORBG_WAVE + lane;
        real[j] = i < n;
        const uint32_t mag = real[j] ? (__float_as_uint(x[j]) & 0x7fffffffu) : 0x7fffffffu;
        key[j] = ((mag >> (IB - 1)) << IB) | (uint32_t)i;
    }
    uint32_t t = guess >> (IB - 1), lo = 0, hi = PMAX, cnt = 0;   // guess: IEEE bits of a magnitude
    bool ok = false;
    for (int it = 0; it < 8; ++it) {
        cnt = 0;
#pragma unroll
        for (int j = 0; j < NK; ++j) cnt += (uint32_t)__builtin_popcountll(ballot(real[j] && (key[j] >> IB) < t));
        if (cnt >= (uint32_t)ra && cnt <= 32u) { ok = true; break; }
        // one binade up or down until the window is bracketed, then bisection
        if (cnt < (uint32_t)ra) {
            lo = t;
            t = (hi == PMAX) ? (t < PMAX - OCT ? t + OCT : PMAX - 1) : lo + (hi - lo) / 2;
        } else {
            hi = t;
            t = (lo == 0) ? (t > OCT ? t - OCT : t / 2) : lo + (hi - lo) / 2;
        }
        t = uniform_u32(t);
    }
    if (!ok) return false;
    // gather: keys below t to LDS slots 0..cnt-1 (T is rebuilt afterwards)
    uint32_t* stage = reinterpret_cast<uint32_t*>(L.T);
    uint32_t base = 0;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const bool c = real[j] && (key[j] >> IB) < t;
        const uint64_t m = ballot(c);
        const uint32_t slot =
            base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (c) stage[slot] = key[j];
        base += (uint32_t)__builtin_popcountll(m);
    }
    wave_lds_sync();
    uint32_t k1[1] = {(uint32_t)lane < cnt ? stage[lane] : 0xffffffffu};
    wave_lds_sync();
    bitonic_sort32_groups<32>(k1);
    const uint32_t next = (uint32_t)__shfl_down((int)k1[0], 1, ORBG_WAVE);
    const bool tie = lane < ra && (uint32_t)lane + 1 < cnt && ((k1[0] ^ next) >> IB) == 0u;
    if (ballot(tie) != 0ull) return false;
    idx1 = k1[0] & ((1u << IB) - 1u);
    // next block's guess: just above the middle of the window
    const uint32_t mid = cnt > 22u ? 22u : (cnt > 0u ? cnt - 1u : 0u);
    const uint32_t g = ((uint32_t)__builtin_amdgcn_readlane((int)k1[0], (int)mid) >> IB) + 1u;
    guess = uniform_u32((g < PMAX ? g : PMAX - 1) << (IB - 1));
    return true;
}

// Per-wave state of the first-batch ranking (wave-uniform).
struct LazyState {
    uint32_t tau;      // threshold guess: IEEE bits of a magnitude
    uint32_t score;    // ~256 x recent rate of blocks decided by the first batch
    uint32_t tries;    // blocks that needed a search
};

// Tables for the first batch after rank_first, in two parts.  first_ranks:
// h[r], pi[r] for r <= ra, and hs[e] = h_{e+1} for the ranks the low-rank
// table covers (read from the lanes that hold them).
template <typename S>
__device__ __forceinline__ void first_ranks(uint32_t idx1, int ra, const S* __restrict__ cols, BlockLds<S>& L,
                                            S (&hs)[ORBG_LOW_RANKS])
{
    const int lane = lane_id();
    const S col = cols[lane < ra ? idx1 : 0u];
    const S hv = lane < ra ? col : (S)0;
    if (lane < ra) {
        L.h[lane + 1] = hv;
        L.pi[lane + 1] = (uint16_t)idx1;
    }
    if (lane == 0) { L.h[0] = 0; L.pi[0] = 0; }
#pragma unroll
    for (int e = 0; e < ORBG_LOW_RANKS; ++e) hs[e] = readlane_s<S>(hv, e);
}

// low_table: T[m] = s0 XOR (XOR of h_r over the bits r - 1 of m), m < 256.
template <typename S>
__device__ __forceinline__ void low_table(const S (&hs)[ORBG_LOW_RANKS], S s0, BlockLds<S>& L)
{
    const int lane = lane_id();
    S a = s0;
#pragma unroll
    for (int b = 0; b < 6; ++b) a ^= ((lane >> b) & 1) ? hs[b] : (S)0;
    L.T[lane] = a;
    L.T[lane + 64] = a ^ hs[6];
    L.T[lane + 128] = a ^ hs[7];
    L.T[lane + 192] = a ^ hs[6] ^ hs[7];
    wave_lds_sync();
}

// Step 3: reliability order and the per-block lookup tables: h[r] = column of
// rank r and pi[r] = its received index for the ranks the schedule reaches,
// T[m] = s0 XOR (XOR of h_r over the bits r - 1 of m) for the 256 subsets of
// ranks 1..8 (h_1..h_8 taken from the lanes that hold them).  FIT: returns the
// block's 1-line offset J0 (fit_offset), else 0.
template <int NK, typename S, bool FIT = false>
__device__ __forceinline__ int rank_and_tables(const float (&x)[NK], int n, const S* __restrict__ cols, S s0,
                                               int rdepth, BlockLds<S>& L)
{
    const int lane = lane_id();
    uint32_t idx[NK];
    rank_order<NK>(x, n, rdepth, FIT ? n / 2 : 0, idx);
    const int j0 = FIT ? fit_offset<NK>(x, idx, n) : 0;
    S hv[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int e = lane * NK + j;          // rank e + 1
        const S col = cols[e < rdepth ? idx[j] : 0u];
        hv[j] = e < rdepth ? col : (S)0;
        if (e < rdepth) {
            L.h[e + 1] = hv[j];
            L.pi[e + 1] = (uint16_t)idx[j];
        }
    }
    if (lane == 0) { L.h[0] = 0; L.pi[0] = 0; }
    S hs[ORBG_LOW_RANKS];
#pragma unroll
    for (int e = 0; e < ORBG_LOW_RANKS; ++e) hs[e] = readlane_s<S>(hv[e % NK], e / NK);
    S a = s0;
#pragma unroll
    for (int b = 0; b < 6; ++b) a ^= ((lane >> b) & 1) ? hs[b] : (S)0;
    L.T[lane] = a;
    L.T[lane + 64] = a ^ hs[6];
    L.T[lane + 128] = a ^ hs[7];
    L.T[lane + 192] = a ^ hs[6] ^ hs[7];
    wave_lds_sync();
    return j0;
}

// Step 4, one step: syndrome of every lane's entry.  Slots past the entry's
// ranks hold rank 0, whose column is zero: the low-rank table and the first
// three slots are read together (one LDS round trip), the last four only when
// some lane's entry has more than three ranks above 8 (a ballot).
// a ^ b ^ c in one instruction (gfx950's three-input bit operation; the
// truth table of a three-way XOR is 0x96).
template <typename S>
__device__ __forceinline__ S xor3(S a, S b, S c);
template <>
__device__ __forceinline__ uint32_t xor3<uint32_t>(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
template <>
__device__ __forceinline__ uint64_t xor3<uint64_t>(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0x96);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0x96);
    return ((uint64_t)hi << 32) | lo;
}

template <typename S>
__device__ __forceinline__ S entry_syndrome(const BlockLds<S>& L, uint2 ent)
{
    const S v0 = L.T[ent.x & 0xffu];
    const S v1 = L.h[(ent.x >> 8) & 0xffu];
    const S v2 = L.h[(ent.x >> 16) & 0xffu];
    const S v3 = L.h[ent.x >> 24];
    S v = xor3<S>(v0, v1, v2) ^ v3;
    if (ballot(ent.y != 0u) != 0ull) {
        const S w0 = L.h[ent.y & 0xffu], w1 = L.h[(ent.y >> 8) & 0xffu];
        const S w2 = L.h[(ent.y >> 16) & 0xffu], w3 = L.h[ent.y >> 24];
        v = xor3<S>(xor3<S>(v, w0, w1), w2, w3);
    }
    return v;
}

// Two steps' syndromes: both entries' first four table reads go out together,
// then one ballot decides whether either needs its last four slots.
template <typename S>
__device__ __forceinline__ void entry_syndrome2(const BlockLds<S>& L, uint2 ea, uint2 eb, S& va, S& vb)
{
    const S a0 = L.T[ea.x & 0xffu], a1 = L.h[(ea.x >> 8) & 0xffu], a2 = L.h[(ea.x >> 16) & 0xffu],
            a3 = L.h[ea.x >> 24];
    const S b0 = L.T[eb.x & 0xffu], b1 = L.h[(eb.x >> 8) & 0xffu], b2 = L.h[(eb.x >> 16) & 0xffu],
            b3 = L.h[eb.x >> 24];
    va = xor3<S>(a0, a1, a2) ^ a3;
    vb = xor3<S>(b0, b1, b2) ^ b3;
    if (ballot((ea.y | eb.y) != 0u) != 0ull) {
        const S c0 = L.h[ea.y & 0xffu], c1 = L.h[(ea.y >> 8) & 0xffu];
        const S c2 = L.h[(ea.y >> 16) & 0xffu], c3 = L.h[ea.y >> 24];
        const S d0 = L.h[eb.y & 0xffu], d1 = L.h[(eb.y >> 8) & 0xffu];
        const S d2 = L.h[(eb.y >> 16) & 0xffu], d3 = L.h[eb.y >> 24];
        va = xor3<S>(xor3<S>(va, c0, c1), c2, c3);
        vb = xor3<S>(xor3<S>(vb, d0, d1), d2, d3);
    }
}

// Step 5: the hard decision with the winning entry's ranks flipped, stored
// through the row's buffer descriptor (lanes past n store nothing).  The
// received position of each flipped rank is wave-uniform: it goes into a
// wave-uniform mask of the positions to flip (one 64-bit word per key), which
// every lane applies once at the end.
template <int NK, typename S, class LO>
__device__ __forceinline__ void write_codeword(const bool (&ybit)[NK], const BlockLds<S>& L, uint32_t win_lo,
                                               uint32_t win_hi, buf_t cw_row, const LO& lo)
{
    const int lane = lane_id();
    uint64_t fm[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) fm[j] = 0;
    auto flip = [&](uint32_t r) {
        const uint32_t p = uniform_u32(L.pi[r]);
        const uint64_t b = 1ull << (p & 63u);
#pragma unroll
        for (int j = 0; j < NK; ++j) fm[j] ^= (p >> 6) == (uint32_t)j ? b : 0ull;
    };
    for (uint32_t low = win_lo & 0xffu; low != 0; low &= low - 1) flip((uint32_t)__builtin_ctz(low) + 1u);
#pragma unroll
    for (int u = 1; u <= ORBG_HIGH_SLOTS; ++u) {
        const uint32_t r = (u < 4) ? ((win_lo >> (8 * u)) & 0xffu) : ((win_hi >> (8 * (u - 4))) & 0xffu);
        if (r != 0) flip(r);
    }
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const uint32_t v = (uint32_t)(ybit[j] ? 1 : 0) ^ (uint32_t)((fm[j] >> lane) & 1ull);
        if constexpr (has_offs<LO>())
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, cw_row, lo.c[j], 0, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, cw_row, j * ORBG_WAVE + lane, 0, 0);
    }
}

// Query count and abandon flag of one block: lane 0's stores are the only ones
// inside the 8-byte and 1-byte descriptors.
__device__ __forceinline__ void write_result(uint64_t* q_out, uint8_t* ab_out, uint32_t q, bool abandon)
{
    const int lane = lane_id();
    const u32x2_t v = {q, 0u};
    __builtin_amdgcn_raw_buffer_store_b64(v, make_buf(q_out, 8), lane * 8, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(abandon ? 1 : 0), make_buf(ab_out, 1), lane, 0, 0);
}

// The same with the kernel's lane offset r (0 on lane 0 only).
__device__ __forceinline__ void write_result(uint64_t* q_out, uint8_t* ab_out, uint32_t q, bool abandon, uint32_t r)
{
    const u32x2_t v = {q, 0u};
    __builtin_amdgcn_raw_buffer_store_b64(v, make_buf(q_out, 8), r, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(abandon ? 1 : 0), make_buf(ab_out, 1), r, 0, 0);
}

// Schedule of a 1-line block with fitted offset j0 (offsets above the code's
// j0max share its last schedule, which orders the first slen patterns alike).
__device__ __forceinline__ const uint2* oneline_schedule(const CodeDesc& c, int j0)
{
    const int jc = j0 < c.j0max ? j0 : c.j0max;
    return c.sched + (size_t)(jc + 1) * c.sstride;
}

// The 1-line offset of one block: lane 0's store is the only one inside the
// 4-byte descriptor.
__device__ __forceinline__ void write_offset(int32_t* j0_out, int j0)
{
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)j0, make_buf(j0_out, 4), lane_id() * 4, 0, 0);
}

// Light pass, one block.  Returns true if the block is left for the heavy pass
// (then nothing is written but the 1-line offset).  ONELINE: the block's fitted
// offset (written to j0_out when that is not null) picks its schedule.  PAIRS:
// the search tests two steps per branch.
template <int NK, bool ORDERED, typename S, bool ONELINE, bool PAIRS, class LO>
__device__ __forceinline__ bool light_block(
    const float (&x)[NK], const uint64_t (&hrow)[NK], const CodeDesc& c, const S* __restrict__ cols,
    BlockLds<S>& L, uint32_t budget, uint32_t split_steps, uint32_t ordv, buf_t cw_row,
    uint64_t* __restrict__ q_out, uint8_t* __restrict__ ab_out, LazyState& lazy, int32_t* __restrict__ j0_out,
    const LO& lo, uint32_t t0 = 0)
{
    const int lane = lane_id();
    const int n = c.n;
    bool ybit[NK];
    const S s0 = hard_decision<NK, S>(x, n, hrow, ybit);

    bool found = false;
    uint32_t q = budget;
    uint32_t win_lo = 0, win_hi = 0;     // winning entry (wave-uniform)

    // 1-line: patterns 2 and 3 are {1} and {2} whatever the offset (J0 w + W
    // orders them right after the empty pattern for every J0 >= -1), so they are
    // tested on ranks 1 and 2 alone, found without sorting the block; the same
    // per-wave score as the basic first-batch ranking (here: how often one of
    // them decides) turns the attempt off while it rarely pays.  Not when the
    // offsets are asked for.
    const uint2* __restrict__ sched = c.sched;
    bool early = false;
    if (ONELINE && s0 != 0 && j0_out == nullptr && n >= 2 && budget >= 3u) {
        lazy.tries = uniform_u32(lazy.tries + 1u);
        uint32_t idx1 = 0;
        if ((lazy.score >= 96u || (lazy.tries & 7u) == 0u) && rank_first<NK, S>(x, n, 2, lazy.tau, L, idx1)) {
            const uint32_t i1 = uniform_u32((uint32_t)__builtin_amdgcn_readlane((int)idx1, 0));
            const uint32_t i2 = uniform_u32((uint32_t)__builtin_amdgcn_readlane((int)idx1, 1));
            const S h1 = cols[i1], h2 = cols[i2];
            if (s0 == h1 || s0 == h2) {
                early = true;
                found = true;
                q = s0 == h1 ? 2u : 3u;
                win_lo = s0 == h1 ? 1u : 2u;          // mask of ranks 1..8: rank 1 or rank 2
                if (lane == 0) {
                    L.pi[1] = (uint16_t)i1;
                    L.pi[2] = (uint16_t)i2;
                }
                wave_lds_sync();
            }
            lazy.score = uniform_u32(lazy.score - (lazy.score >> 3) + (early ? 32u : 0u));
        }
    }
    // otherwise the offset needs the whole ranking, made here when the block
    // needs a search or its offset is asked for
    if (ONELINE && !early && (s0 != 0 || j0_out != nullptr)) {
        const int j0 = rank_and_tables<NK, S, true>(x, n, cols, s0, c.rdepth, L);
        if (j0_out != nullptr) write_offset(j0_out, j0);
        sched = oneline_schedule(c, j0);
    }

    // s0 == 0: the empty pattern (entry 0 of batch 0) is a member; it is the first
    // hit when batch 0 is tested first (always in the plain and 1-line orders)
    if (early) {
        // decided by {1} or {2}
    } else if (s0 == 0 && (!ORDERED || batch_at<ORDERED>(ordv, 0) == 0)) {
        found = true;
        q = 1;
    } else {
        const uint32_t slen = c.slen;
        // Step t tests batch bt; lane l takes schedule entry 64 bt + l, which is
        // query number 64 t + l + 1.  The queries that exist are the first
        // lim = min(budget, schedule length), so there are T steps and only the
        // last one masks lanes.  Indices fit 32 bits.
        const uint32_t lim = min(budget, slen);
        const uint32_t T = (lim + ORBG_WAVE - 1) / ORBG_WAVE;
        // entries of step u: a schedule holds whole batches of 64 entries and
        // ORBG_SCHED_PAD zero batches after its last one, so the loads for up to
        // five steps past the end stay inside it and need no bounds check
        auto entries = [&](uint32_t u) -> uint2 {
            return load_entry(sched, batch_at<ORDERED>(ordv, u) * ORBG_WAVE + (uint32_t)lane);
        };
        // the first three (PAIRS: four) steps' entries do not depend on the
        // block's order of reliability: they load while the ranks are sorted
        // (1-line: after the ranking that picks the schedule)
        // (t0 = 1: batch 0 is known to hold no member and is counted, not tested)
        uint2 e0 = entries(t0), e1 = entries(t0 + 1), e2 = entries(t0 + 2);
        uint2 e3 = PAIRS ? entries(t0 + 3) : make_uint2(0u, 0u);
        uint32_t t = t0;
        // the search stops at step tend: the end of the queries, or the split
        // point if that comes first
        const uint32_t tend = (split_steps != 0 && split_steps < T) ? split_steps : T;
        // The search state is t, the steps left before tend and the ballot of
        // the hits of the step that ended it: a step function returns true when
        // the search stops (a hit, or step tend reached).
        uint64_t hits = 0;
        uint32_t rem = tend > t0 ? tend - t0 : 0u;
        // One step: load the entries of step t + 3, test those of step t, move
        // to step t + 1.  Four register sets rotate, so a load is consumed
        // three steps after it was issued.
        auto step = [&](const uint2 cur, uint2& ahead) -> bool {
            ahead = entries(t + 3);
            hits = ballot(entry_syndrome<S>(L, cur) == 0);
            ++t;
            --rem;
            return hits != 0 || rem == 0;
        };
        // PAIRS: steps t and t + 1 under one branch (a hit in step t comes
        // first; step t + 1 counts only if it lies before tend), their eight
        // table reads out together, and the pair's registers then take the
        // entries of steps t + 4 and t + 5: half the scalar bookkeeping per
        // step.  It needs a few more registers, so only the kernels that have
        // them use it (one code, two keys per lane).
        auto pair = [&](uint2& ea, uint2& eb, uint64_t& ha, uint64_t& hb) {
            S va, vb;
            entry_syndrome2<S>(L, ea, eb, va, vb);
            // the pair's registers take steps t + 4 and t + 5 once read
            ea = entries(t + 4);
            eb = entries(t + 5);
            ha = ballot(va == 0);
            hb = ballot(vb == 0);
        };
        // 0 (go on), 1 (hit), 2 (no hit within the budget), 3 (split point).
        // Only the last step of the queries holds lanes past the budget (query
        // numbers above lim): a first hit there means no hit within the budget,
        // so no lane mask is carried from step to step.  The winning entry is
        // read again (one scalar load) rather than kept from the step.
        auto outcome = [&](bool stop) -> int {
            if (!stop) return 0;
            if (hits) {                               // found in step t - 1
                const uint32_t wl = (uint32_t)__builtin_ctzll(hits);
                q = (t - 1) * ORBG_WAVE + wl + 1;
                if (q > lim) return 2;
                const uint32_t* w =
                    reinterpret_cast<const uint32_t*>(sched + batch_at<ORDERED>(ordv, t - 1) * ORBG_WAVE + wl);
                win_lo = scalar_load(w, 0);
                win_hi = scalar_load(w, 1);
                return 1;
            }
            return t * ORBG_WAVE >= lim ? 2 : 3;
        };
        // Plain order: most blocks end in the first batch, which only reaches
        // ranks 1..rdepth0, so those ranks are found first (rank_first) and the
        // first step runs on them; the whole block is ranked only if it goes on.
        // Whether to try: a per-wave score of how often the first batch decided
        // (decays by 1/8 per try, +32 per success, so it tends to 256 x the
        // success rate); below 5/8 it pays to rank the whole block at once, but
        // every 8th block still tries so that the score follows the channel.
        // A search that stops after step 0 (split_steps = 1) always tries: it
        // never needs more ranks than the first batch reaches.
        int r = 0;
        bool resume = false;                  // step 0 already tested (one-step loop)
        uint32_t idx1 = 0;
        lazy.tries = uniform_u32(lazy.tries + 1u);
        if (!ORDERED && !ONELINE && (lazy.score >= 160u || (lazy.tries & 7u) == 0u || split_steps == 1u) &&
            rank_first<NK, S>(x, n, c.rdepth0, lazy.tau, L, idx1)) {
            S hs[ORBG_LOW_RANKS];
            first_ranks<S>(idx1, c.rdepth0, cols, L, hs);
            low_table<S>(hs, s0, L);
            if constexpr (PAIRS) {
                // step 0 alone; the entries move down one step, the next load
                // taking step 4
                const uint2 e4 = entries(t + 4);
                hits = ballot(entry_syndrome<S>(L, e0) == 0);
                ++t;
                --rem;
                r = outcome(hits != 0 || rem == 0);
                e0 = e1;
                e1 = e2;
                e2 = e3;
                e3 = e4;
            } else {
                r = outcome(step(e0, e3));
                resume = true;
            }
            lazy.score = uniform_u32(lazy.score - (lazy.score >> 3) + (r != 0 ? 32u : 0u));
        }
        if (r == 0 && rem == 0) r = outcome(true);          // nothing left to test after batch 0
        if (r == 0) {
            if (!ONELINE) rank_and_tables<NK, S>(x, n, cols, s0, c.rdepth, L);
            if constexpr (PAIRS) {
                // the loop moves on while neither step hit and more than two
                // steps are left (one scalar test); the pair that stops it is
                // settled after it
                // (rem - 3) >> 31 is rem <= 2 (rem < 2^31) as a bit: computed
                // without a compare, the test stays on the scalar unit
                uint64_t ha, hb;
                for (;;) {
                    pair(e0, e1, ha, hb);
                    if ((ha | hb | (uint64_t)((rem - 3u) >> 31)) != 0) break;
                    t += 2;
                    rem -= 2;
                    pair(e2, e3, ha, hb);
                    if ((ha | hb | (uint64_t)((rem - 3u) >> 31)) != 0) break;
                    t += 2;
                    rem -= 2;
                }
                const uint32_t adv = (ha != 0 || rem == 1) ? 1u : 2u;
                hits = adv == 1u ? ha : hb;
                t += adv;
                rem -= adv;
            } else {
                for (;;) {
                    if (!resume && step(e0, e3)) break;
                    resume = false;
                    if (step(e1, e0)) break;
                    if (step(e2, e1)) break;
                    if (step(e3, e2)) break;
                }
            }
            r = outcome(true);
        }
        // the entries prefetched for steps that will not run are taken here, so
        // their registers are free when the next block's code reuses them (no
        // wait on the next block's row at the top of the block loop)
        asm volatile("" ::"v"(e0.x), "v"(e0.y), "v"(e1.x), "v"(e1.y), "v"(e2.x), "v"(e2.y), "v"(e3.x),
                     "v"(e3.y));
        if (r == 3) {
            wave_lds_sync();
            return true;
        }
        found = (r == 1);
    }

    write_codeword<NK, S>(ybit, L, win_lo, win_hi, cw_row, lo);
    if constexpr (has_offs<LO>())
        write_result(q_out, ab_out, found ? q : budget, !found, lo.r);
    else
        write_result(q_out, ab_out, found ? q : budget, !found);
    wave_lds_sync();
    return false;
}

template <int NK, bool ORDERED, typename S, bool ONELINE, bool PAIRS = false, class LO = NoOffs>
__device__ __forceinline__ void light_one(const float (&x)[NK], const uint64_t (&hrow)[NK], uint32_t ordv,
                                          const CodeDesc& c, const S* cols, BlockLds<S>& L, int64_t b, int64_t row,
                                          uint32_t budget, uint32_t split_steps, uint8_t* cw, uint64_t* queries,
                                          uint8_t* abandoned, unsigned long long* ctrs, int64_t* heavy,
                                          LazyState& lazy, int32_t* j0_out, uint32_t t0, const LO& lo)
{
    const bool left = light_block<NK, ORDERED, S, ONELINE, PAIRS, LO>(
        x, hrow, c, cols, L, budget, split_steps, ordv,
        make_buf(cw + (row >= 0 ? row : 0), row >= 0 ? (uint32_t)c.n : 0u), queries + b, abandoned + b, lazy,
        j0_out ? j0_out + b : nullptr, lo, t0);
    if (left && lane_id() == 0) {
        const unsigned long long slot = atomicAdd(ctrs + ORBG_CTR_HEAVY_COUNT, 1ull);
        heavy[slot] = b;
    }
}

// Next block's inputs, fetched while the current block is decoded.
template <int NKMAX>
struct RowFetch {
    float x[NKMAX];
    int64_t oid;       // index of the block's outputs (wave-uniform)
    uint32_t ordv;     // batch order (ordered decode)
    int ci;            // code index (wave-uniform)
    int64_t row;       // element offset of the row (wave-uniform)
};

// Byte `i` of a read-only array, by a scalar load of its dword.
__device__ __forceinline__ uint32_t scalar_load_u8(const uint8_t* p, int64_t i)
{
    const uintptr_t a = (uintptr_t)(p + i);
    return (scalar_load((const uint32_t*)(a & ~(uintptr_t)3), 0) >> ((a & 3) * 8)) & 0xffu;
}

__device__ __forceinline__ int64_t scalar_load_i64(const int64_t* p, int64_t i)
{
    const uint32_t* w = (const uint32_t*)(p + i);
    return (int64_t)(((uint64_t)scalar_load(w, 1) << 32) | scalar_load(w, 0));
}

// Rows of H for this lane padded to NK words (words past the code's nk are zero).
template <int NK>
__device__ __forceinline__ void load_hrows_pad(const uint64_t* rows, int m, int nk, uint64_t (&h)[NK])
{
    const int r = lane_id() < m ? lane_id() : 0;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const uint64_t w = j < nk ? rows[r * nk + j] : 0ull;
        h[j] = lane_id() < m ? w : 0ull;
    }
}

// Rows in flight per screening group: 16 row registers per lane.
template <int NKMAX>
struct ScreenDepth { static constexpr int value = NKMAX >= 16 ? 1 : 16 / NKMAX; };

// Light pass.  One wave per workgroup, so the wave's LDS tables sit at fixed
// addresses.  MIXED: each block names its code (block_code) and row offset;
// otherwise all blocks use code 0 with rows b * n.  NKMAX: largest keys per
// lane among the launch's codes.
//
// Each wave takes chunks of `chunk` (at most 64) consecutive blocks from the
// counters of 64 work slices (striped over the batch; workgroup w works first
// on slice w % 64, which lies on its own XCD, then helps the other slices;
// the work cursor below); the counter increment for the next chunk is issued
// when a chunk starts.  A chunk is decoded in two phases:
//   1. screening: the rows are read K at a time, all K loads in flight
//      together, and every block whose base syndrome is zero (query 1 is a
//      member and comes first) is written out at once;
//   2. the other blocks (a 64-bit mask) are decoded one by one, the next one's
//      row loaded while the current one is decoded; the two fetch buffers
//      alternate, so no register copy waits for a load.
// Waves per SIMD the light pass asks the register allocator for (the device
// holds at most 8, 32 per CU), chosen by measurement with 32-bit syndromes:
// 1 key per lane fits 64 vector registers at 8 waves; 2 keys per lane run
// best at 7 (at 8 some registers go to scratch, at 6 too few waves hide the
// latency), except in 1-line mode (no first-batch ranking), which runs best
// at 8; 4 keys per lane at 6; wider variants keep the compiler's choice.
template <int NKMAX, typename S, bool ONELINE>
constexpr int light_waves()
{
    return sizeof(S) != 4 ? 1 : NKMAX == 1 ? 8 : NKMAX == 2 ? (ONELINE ? 8 : 7) : NKMAX == 4 ? 6 : 1;
}

template <int NKMAX, bool ORDERED, typename S, bool MIXED, bool ONELINE>
__global__ void __launch_bounds__(ORBG_WAVE) __attribute__((amdgpu_waves_per_eu(light_waves<NKMAX, S, ONELINE>())))
light_kernel(CodeTable codes, const uint8_t* __restrict__ block_code, const int64_t* __restrict__ row_off,
             const float* __restrict__ llr, int64_t nblocks, uint32_t budget, uint32_t split_steps,
             const uint8_t* __restrict__ order, uint8_t* __restrict__ cw, uint64_t* __restrict__ queries,
             uint8_t* __restrict__ abandoned, unsigned long long* __restrict__ ctrs, int64_t* __restrict__ heavy,
             int chunk, int32_t* __restrict__ j0_out, int64_t row_limit, const int64_t* __restrict__ ids,
             uint32_t t0, int naive, uint32_t fixed)
{
    // dynamic LDS (sized at launch): the rows of the launch's codes (sum of
    // m x nk words), then their columns (sum of n entries)
    extern __shared__ __align__(16) unsigned char orbg_dyn_lds[];
    uint64_t* s_rows = reinterpret_cast<uint64_t*>(orbg_dyn_lds);
    S* s_cols = reinterpret_cast<S*>(orbg_dyn_lds + (size_t)codes.rwords * sizeof(uint64_t));
    __shared__ BlockLds<S> L;
    for (int ci = 0; ci < (MIXED ? codes.ncodes : 1); ++ci) {
        const CodeDesc& c = codes.c[ci];
        for (int i = threadIdx.x; i < c.n; i += ORBG_WAVE) s_cols[c.col_base + i] = (S)c.cols[i];
        for (int i = threadIdx.x; i < c.m * c.nk; i += ORBG_WAVE) s_rows[c.row_base + i] = c.rows[i];
    }
    wave_lds_sync();
    const int lane = lane_id();
    // rank_first's threshold (start at |LLR| = 2) and try policy, carried from
    // block to block
    LazyState lazy = {0x40000000u, 256u, 0u};
    // one code with at most 4 words per row: the rows stay in registers
    constexpr bool HOIST = !MIXED && NKMAX <= 4;
    uint64_t hrow0[NKMAX];
    if (HOIST) load_hrows<NKMAX>(s_rows, codes.c[0].m, hrow0);
    // One code with two keys per lane (the kernel of the widest use): every row
    // and result access takes its lane offsets from one set made here, lanes
    // past n cut, and the screening reads a group's rows through one
    // descriptor.  The other kernels compute lane offsets in place (a kernel-wide
    // set spilled registers there).
    constexpr bool FLAT = !MIXED && NKMAX == 2;
    using LO = typename std::conditional<FLAT, LaneOffs<NKMAX>, NoOffs>::type;
    LO lo;
    if constexpr (FLAT) lo = lane_offsets<NKMAX>(codes.c[0].n);

    // Work cursor (wave-uniform).  The blocks are dealt to ORBG_SLICES slices in
    // stripes of Z blocks: stripe g (blocks [g Z, (g + 1) Z)) goes to slice
    // g % S, so every slice holds the same mix of the batch (a batch laid out by
    // channel condition still gives slices of equal cost, which drain
    // together).  Z is a whole number of chunks, up to ORBG_STRIPE of them, and
    // small enough that each slice gets about 8 stripes or more.  Workgroup w
    // starts on slice w % S, which lies on its own XCD (workgroups are dealt
    // round-robin to the 8 XCDs).  A slice's counter counts the blocks claimed,
    // `chunk` at a time (chunks never cross a stripe, Z being a multiple of the
    // chunk); `pend` (lane 0) receives the next chunk's counter value, claimed
    // when a chunk starts.  Increments of one counter queue one behind another
    // (of the order of 0.1 us each), so many slices keep few waves on each
    // counter: with one slice per XCD, the increments that find slices drained
    // cost about 0.1 ms per launch, whatever the number of blocks.
    const int64_t zc = nblocks / ((int64_t)ORBG_SLICES * chunk * 8);
    const int64_t Z = (int64_t)chunk * (zc < 1 ? 1 : zc > ORBG_STRIPE ? ORBG_STRIPE : zc);
    const int64_t nstripes = (nblocks + Z - 1) / Z;
    // blocks in slice x: stripes x, x + S, ... (the batch's last stripe may be short)
    auto slice_len = [&](int64_t x) -> int64_t {
        if (x >= nstripes) return 0;
        const int64_t cnt = (nstripes - 1 - x) / ORBG_SLICES + 1;
        const int64_t last = (x + (cnt - 1) * ORBG_SLICES) * Z;
        return (cnt - 1) * Z + (nblocks - last < Z ? nblocks - last : Z);
    };
    const int home = (int)(blockIdx.x % ORBG_SLICES);
    int slice = home;
    int64_t len = uniform_i64(slice_len(home)), end = 0;
    unsigned long long* ctr = ctrs + ORBG_CTR_SLICE(home);
    // The first chunk of each of the first `fixed` workgroups of a slice
    // (those resident from the start) is fixed, with no increment: workgroup w
    // is the (w / S)-th of its slice and takes that chunk of it, and the
    // counters start past those chunks (set so before the launch).  Otherwise
    // every wave would start by queueing on its slice's counter, the last of a
    // slice's waves ~0.1 us x their number later.  Later workgroups (they start
    // only as others end) claim their first chunk as usual.
    const uint32_t rank = blockIdx.x / ORBG_SLICES;
    unsigned long long pend = (unsigned long long)rank * (unsigned long long)chunk;
    if (rank >= fixed && lane == 0) pend = atomicAdd(ctr, (unsigned long long)chunk);
    // The slice to move to when the current one is drained, or -1 when all are:
    // lane x reads slice x's counter (one coherent load, no increment), and
    // since a counter only grows, a slice seen drained stays drained.  The pick
    // is the nearest open slice after the home slice on the same XCD, else the
    // nearest open one (bit j of rot: slice (home + j) % S; j a multiple of 8:
    // the same XCD).
    auto next_open = [&]() -> int {
        static_assert(ORBG_SLICES == ORBG_WAVE, "one lane per slice");
        static_assert(ORBG_XCDS == 8, "slices of one XCD are 8 apart");
        const unsigned long long v =
            __hip_atomic_load(ctrs + ORBG_CTR_SLICE(lane), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t rot = __builtin_rotateright64(ballot((int64_t)v < slice_len(lane)), (unsigned)home);
        if (rot == 0) return -1;
        constexpr uint64_t SAME_XCD = 0x0101010101010101ull;
        const uint64_t pick = (rot & SAME_XCD) != 0 ? (rot & SAME_XCD) : rot;
        return (int)uniform_u32((uint32_t)((home + __builtin_ctzll(pick)) % ORBG_SLICES));
    };
    // first block of the next chunk (its end in `end`), or -1 when every slice
    // is drained.  Every cursor value goes through readfirstlane so that it
    // stays in scalar registers and the branches on it stay scalar.  Each failed
    // increment leaves its slice seen drained by the next snapshot, so the loop
    // ends after at most ORBG_SLICES of them.
    auto next_chunk = [&]() -> int64_t {
        int64_t s;
        for (;;) {
            const int64_t p = uniform_i64((int64_t)uniform_u64(pend));
            const bool hit = p < len;
            if (hit) {
                s = uniform_i64((p / Z * ORBG_SLICES + slice) * Z + p % Z);
                end = uniform_i64(s + (len - p < chunk ? len - p : chunk));
            } else {
                slice = next_open();
                if (slice < 0) return -1;
                len = uniform_i64(slice_len(slice));
                ctr = ctrs + ORBG_CTR_SLICE(slice);
            }
            // one lane increments; the loop leaves only after this branch has joined
            if (lane == 0) pend = atomicAdd(ctr, (unsigned long long)chunk);
            if (hit) break;
        }
        return s;
    };
    // code index, row offset and output index of the launch's b-th block
    // (wave-uniform).  Mixed launches: a row that does not lie inside the first
    // row_limit elements of both the LLR and the codeword buffer gets row = -1:
    // it is read as zeros and its codeword stores are dropped (its queries and
    // flag are still written).  A block list (ids) names the caller's block of
    // each position: its row, codeword and outputs; the batch order is the
    // list's own (row b).
    auto locate = [&](int64_t b, int& ci, int64_t& row, int64_t& oid) {
        if (MIXED) {
            ci = (int)scalar_load_u8(block_code, b);
            ci = ci < codes.ncodes ? ci : 0;          // out-of-range indices read code 0
            row = scalar_load_i64(row_off, b);
            row = uniform_i64((row >= 0 && row <= row_limit - codes.c[ci].n) ? row : -1);
            oid = b;
        } else {
            ci = 0;
            oid = ids ? scalar_load_i64(ids, b) : b;
            row = oid * codes.c[0].n;
        }
    };

    // phase 1 over [s, e): returns the mask (bit b - s) of the blocks left
    constexpr int K = ScreenDepth<NKMAX>::value;
    auto screen = [&](int64_t s, int64_t e) -> uint64_t {
        uint64_t left = 0;
        if constexpr (!MIXED) {
            // One code: nothing per row is held across the loads but the
            // fetched values.  A row's output index and offset are computed
            // again from the group start when it is screened (the group start
            // and row count pass through an empty asm statement, so the two
            // computations stay apart): held, the K offsets and their masks
            // exceed the scalar registers, and their spills to vector lanes
            // cost more vector instructions than the screening itself.
            const CodeDesc& c = codes.c[0];
            const int n = c.n;
            if constexpr (FLAT) {
                if (ids == nullptr) {
                    // Blocks in launch order: a group's rows lie back to back, so
                    // one descriptor covers them all (and one each the group's
                    // codewords, query counts and flags) and a row is picked by a
                    // scalar offset, the only per-row address arithmetic.  Lanes
                    // past n hold offsets beyond every descriptor's size (lo), so
                    // they read 0 and their stores are dropped whether or not the
                    // scalar offset enters the hardware's range check; rows past
                    // the group's count take scalar offset 0 (a row of the group,
                    // read and never screened).
                    const uint32_t n4 = (uint32_t)n * 4u;
                    for (int64_t g = s; g < e; g += K) {
                        float xs[K][NKMAX];
                        uint32_t first[K];
                        uint32_t cnt = uniform_u32((uint32_t)((e - g) < K ? (e - g) : K));
                        asm volatile("" : "+s"(cnt));     // compared as a 32-bit scalar below
                        const buf_t lb = make_buf(llr + g * n, cnt * n4);
                        const buf_t ob = make_buf(ORDERED ? order + g * 64 : order, ORDERED ? cnt * 64u : 0u);
#pragma unroll
                        for (int kk = 0; kk < K; ++kk) {
                            const bool ok = (uint32_t)kk < cnt;
                            load_row_buf<NKMAX>(lb, xs[kk], lo, ok ? (uint32_t)kk * n4 : 0u);
                            first[kk] = ORDERED ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(
                                                      ob, lo.r, ok ? (uint32_t)kk * 64u : 0u, 0)
                                                : 0u;
                        }
                        int64_t g2 = g;
                        uint32_t cnt2 = cnt;
                        asm volatile("" : "+s"(g2), "+s"(cnt2));
                        const buf_t cb = make_buf(cw + g2 * n, cnt2 * (uint32_t)n);
                        const buf_t qb = make_buf(queries + g2, cnt2 * 8u);
                        const buf_t ab = make_buf(abandoned + g2, cnt2);
#pragma unroll
                        for (int kk = 0; kk < K; ++kk) {
                            if ((uint32_t)kk < cnt2) {
                                uint64_t hr[NKMAX];
                                if (HOIST) {
#pragma unroll
                                    for (int j = 0; j < NKMAX; ++j) hr[j] = hrow0[j];
                                } else {
                                    load_hrows<NKMAX>(s_rows, c.m, hr);
                                }
                                bool yb[NKMAX];
                                const S s0 = hard_decision<NKMAX, S>(xs[kk], n, hr, yb);
                                const bool done = s0 == 0 && (!ORDERED || uniform_u32(first[kk]) == 0u) &&
                                                  !(ONELINE && j0_out != nullptr);
                                if (done) {
#pragma unroll
                                    for (int j = 0; j < NKMAX; ++j)
                                        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(yb[j] ? 1 : 0), cb, lo.c[j],
                                                                             (uint32_t)kk * (uint32_t)n, 0);
                                    const u32x2_t q1 = {1u, 0u};
                                    __builtin_amdgcn_raw_buffer_store_b64(q1, qb, lo.r, (uint32_t)kk * 8u, 0);
                                    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)0, ab, lo.r, (uint32_t)kk, 0);
                                } else {
                                    left |= 1ull << (g2 + kk - s);
                                }
                            }
                        }
                    }
                    return left;
                }
            }
            // A block list: each row's output index is read from the list.
            auto out_index = [&](int64_t b) -> int64_t { return ids ? scalar_load_i64(ids, b) : b; };
            for (int64_t g = s; g < e; g += K) {
                float xs[K][NKMAX];
                uint32_t first[K];
                const uint32_t cnt = uniform_u32((uint32_t)((e - g) < K ? (e - g) : K));
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    const bool ok = (uint32_t)kk < cnt;
                    const int64_t oid = ok ? out_index(g + kk) : 0;
                    load_row_buf<NKMAX>(make_buf(llr + oid * n, ok ? (uint32_t)n * 4u : 0u), xs[kk], lo);
                    first[kk] = ORDERED ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(
                                              make_buf(order + (ok ? g + kk : 0) * 64, ok ? 1u : 0u), 0, 0, 0)
                                        : 0u;
                }
                int64_t g2 = g;
                uint32_t cnt2 = cnt;
                asm volatile("" : "+s"(g2), "+s"(cnt2));
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    if ((uint32_t)kk < cnt2) {
                        uint64_t hr[NKMAX];
                        if (HOIST) {
#pragma unroll
                            for (int j = 0; j < NKMAX; ++j) hr[j] = hrow0[j];
                        } else {
                            load_hrows<NKMAX>(s_rows, c.m, hr);
                        }
                        bool yb[NKMAX];
                        const S s0 = hard_decision<NKMAX, S>(xs[kk], n, hr, yb);
                        const bool done = s0 == 0 && (!ORDERED || uniform_u32(first[kk]) == 0u) &&
                                          !(ONELINE && j0_out != nullptr);
                        if (done) {
                            const int64_t oid = out_index(g2 + kk);
                            const buf_t cwr = make_buf(cw + oid * n, (uint32_t)n);
#pragma unroll
                            for (int j = 0; j < NKMAX; ++j) {
                                if constexpr (FLAT)
                                    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(yb[j] ? 1 : 0), cwr, lo.c[j], 0, 0);
                                else
                                    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(yb[j] ? 1 : 0), cwr,
                                                                         j * ORBG_WAVE + lane, 0, 0);
                            }
                            if constexpr (FLAT)
                                write_result(queries + oid, abandoned + oid, 1u, false, lo.r);
                            else
                                write_result(queries + oid, abandoned + oid, 1u, false);
                        } else {
                            left |= 1ull << (g2 + kk - s);
                        }
                    }
                }
            }
            return left;
        }
        for (int64_t g = s; g < e; g += K) {
            float xs[K][NKMAX];
            int cis[K];
            bool use[K];
            int64_t rows[K], oids[K];
            uint32_t first[K];
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                bool ok = g + kk < e;
                int ci = 0;
                int64_t row = 0, oid = 0;
                if (ok) locate(g + kk, ci, row, oid);
                use[kk] = ok;
                cis[kk] = ci;
                rows[kk] = row;
                oids[kk] = oid;
                const bool rv = ok && row >= 0;
                load_row_buf<NKMAX>(make_buf(llr + (rv ? row : 0), rv ? (uint32_t)codes.c[ci].n * 4u : 0u), xs[kk]);
                // ordered decode: the block's first batch (every lane reads byte 0)
                first[kk] = ORDERED ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(
                                          make_buf(order + (ok ? g + kk : 0) * 64, ok ? 1u : 0u), 0, 0, 0)
                                    : 0u;
            }
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                const int64_t b = g + kk;
                if (use[kk]) {
                    const CodeDesc& c = codes.c[cis[kk]];
                    uint64_t hr[NKMAX];
                    if (HOIST) {
#pragma unroll
                        for (int j = 0; j < NKMAX; ++j) hr[j] = hrow0[j];
                    } else {
                        load_hrows_pad<NKMAX>(s_rows + c.row_base, c.m, c.nk, hr);
                    }
                    bool yb[NKMAX];
                    const S s0 = hard_decision<NKMAX, S>(xs[kk], c.n, hr, yb);
                    // (1-line offsets asked for: every block is ranked in phase 2)
                    const bool done = s0 == 0 && (!ORDERED || uniform_u32(first[kk]) == 0u) &&
                                      !(ONELINE && j0_out != nullptr);
                    if (done) {
                        const buf_t cwr = make_buf(cw + (rows[kk] >= 0 ? rows[kk] : 0), rows[kk] >= 0 ? (uint32_t)c.n : 0u);
#pragma unroll
                        for (int j = 0; j < NKMAX; ++j)
                            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(yb[j] ? 1 : 0), cwr, j * ORBG_WAVE + lane,
                                                                 0, 0);
                        write_result(queries + oids[kk], abandoned + oids[kk], 1u, false);
                    } else {
                        left |= 1ull << (b - s);
                    }
                }
            }
        }
        return left;
    };

    // phase 2: the inputs of block b (b < 0: an empty row, every lane reads 0)
    auto fetch = [&](RowFetch<NKMAX>& f, int64_t b) {
        int ci = 0;
        int64_t row = 0, oid = 0;
        if (b >= 0) locate(b, ci, row, oid);
        f.ci = ci;
        f.row = row;
        f.oid = oid;
        const bool rv = b >= 0 && row >= 0;
        const uint32_t bytes = rv ? (uint32_t)codes.c[ci].n * 4u : 0u;
        load_row_buf<NKMAX>(make_buf(llr + (rv ? row : 0), bytes), f.x, lo);
        f.ordv = ORDERED ? load_order_buf(make_buf(order + (b >= 0 ? b : 0) * 64, b >= 0 ? 64u : 0u)) : 0u;
    };
    auto decode = [&](const RowFetch<NKMAX>& f, int64_t b) {
        const CodeDesc& c = codes.c[MIXED ? f.ci : 0];
        const S* cols = s_cols + (MIXED ? c.col_base : 0);
        if (HOIST) {
            light_one<NKMAX, ORDERED, S, ONELINE, !MIXED && NKMAX == 2>(f.x, hrow0, f.ordv, c, cols, L, f.oid, f.row,
                                                                        budget, split_steps, cw, queries, abandoned,
                                                                        ctrs, heavy, lazy, j0_out, t0, lo);
        } else if (!MIXED || NKMAX == 1 || c.nk == NKMAX) {
            uint64_t hr[NKMAX];
            load_hrows<NKMAX>(s_rows + c.row_base, c.m, hr);
            light_one<NKMAX, ORDERED, S, ONELINE>(f.x, hr, f.ordv, c, cols, L, f.oid, f.row, budget, split_steps, cw,
                                                  queries, abandoned, ctrs, heavy, lazy, j0_out, t0, lo);
        } else if (c.nk == 1) {
            uint64_t hr[1];
            load_hrows<1>(s_rows + c.row_base, c.m, hr);
            light_one<1, ORDERED, S, ONELINE>(*reinterpret_cast<const float(*)[1]>(f.x), hr, f.ordv, c, cols, L, f.oid,
                                              f.row, budget, split_steps, cw, queries, abandoned, ctrs, heavy, lazy,
                                              j0_out, t0, NoOffs{});
        } else {
            constexpr int K2 = NKMAX >= 2 ? 2 : 1;
            uint64_t hr[K2];
            load_hrows<K2>(s_rows + c.row_base, c.m, hr);
            light_one<K2, ORDERED, S, ONELINE>(*reinterpret_cast<const float(*)[K2]>(f.x), hr, f.ordv, c, cols, L,
                                               f.oid, f.row, budget, split_steps, cw, queries, abandoned, ctrs, heavy,
                                               lazy, j0_out, t0, NoOffs{});
        }
    };

    // One block per workgroup (the baseline a plain launch gives: no work
    // counter, no chunks, no heavy pass): workgroup b decodes block b.
    if (naive) {
        if ((int64_t)blockIdx.x < nblocks) {
            RowFetch<NKMAX> f;
            fetch(f, (int64_t)blockIdx.x);
            decode(f, (int64_t)blockIdx.x);
        }
        return;
    }
    // phase 2 over the blocks left in [base, base + 64) (bit i: block base + i)
    auto phase2 = [&](uint64_t left, int64_t base) {
        int64_t b = base + __builtin_ctzll(left);
        left &= left - 1;
        RowFetch<NKMAX> fa, fb;
        fetch(fa, b);
        auto advance = [&](const RowFetch<NKMAX>& cur, RowFetch<NKMAX>& nxt) -> bool {
            const int64_t bn = left ? base + __builtin_ctzll(left) : -1;
            left &= left - 1;
            fetch(nxt, bn);
            decode(cur, b);
            b = bn;
            return bn >= 0;
        };
        for (;;) {
            if (!advance(fa, fb)) break;
            if (!advance(fb, fa)) break;
        }
    };
    // One code, two keys per lane, not 1-line: a chunk is worked through K
    // blocks at a time, one screening group and then its phase 2, so the
    // phase-2 rows are read again while the screening's reads of them still sit
    // in L2 (with the whole chunk screened first, most of those reads miss it),
    // the counter still taking one increment per chunk.  The other kernels
    // screen whole chunks: there the extra loop state spilled registers to
    // scratch.
    constexpr bool BY_GROUP = NKMAX == 2 && !ONELINE && !MIXED;
    for (int64_t s = uniform_i64(next_chunk()); s >= 0; s = uniform_i64(next_chunk())) {
        if constexpr (BY_GROUP) {
            for (int64_t g = s; g < end; g += K) {
                const uint64_t left = screen(g, (g + K < end) ? g + K : end);
                if (left != 0) phase2(left, g);
            }
        } else {
            const uint64_t left = screen(s, end);
            if (left != 0) phase2(left, s);
        }
    }
}

// Heavy pass, one block shared by the workgroup's G waves (all waves call it).
// Plain order only: blocks reach it after at least 64 steps or were never reordered.
// ONELINE: wave 0 fits the block's offset again and shares it through *s_j0.
template <int NK, typename S, int G, bool ONELINE>
__device__ __forceinline__ void heavy_block(const CodeDesc& c, const float* __restrict__ llr_row, S* s_cols,
                                            BlockLds<S>& L, uint32_t* best, int* s_j0, uint32_t budget,
                                            uint32_t split_steps, uint8_t* __restrict__ cw_row,
                                            uint64_t* __restrict__ q_out, uint8_t* __restrict__ ab_out, bool row_ok)
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
        load_row<NK>(llr_row, row_ok ? n : 0, x);
        uint64_t hr[NK];
        load_hrows<NK>(c.rows, c.m, hr);
        const S s0 = hard_decision<NK, S>(x, n, hr, ybit);
        const int j0 = rank_and_tables<NK, S, ONELINE>(x, n, s_cols, s0, c.rdepth, L);
        if (ONELINE && lane == 0) *s_j0 = j0;
    }
    __syncthreads();
    const uint2* __restrict__ sched = ONELINE ? oneline_schedule(c, (int)uniform_u32((uint32_t)*s_j0)) : c.sched;
    const uint32_t slen = c.slen;
    // wave w takes steps split + w, split + w + G, ...; the next one's entries
    // are loaded while the current one is tested
    uint32_t t = split_steps + wave;
    const uint32_t lim = min(budget, slen);
    if (t * ORBG_WAVE < lim) {
        uint2 entA = load_entry(sched, min(t * ORBG_WAVE + lane, slen - 1));
        uint2 entB = make_uint2(0u, 0u);
        // returns true when this wave is done (hit, nothing left, or an earlier hit known)
        auto step = [&](const uint2 cur, uint2& nxt) -> bool {
            if (t * ORBG_WAVE + 1 > __hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                return true;
            const uint32_t t1 = t + G;
            const bool has_next = t1 * ORBG_WAVE < lim;
            const uint32_t tl = has_next ? t1 : t;            // loads on every path
            nxt = load_entry(sched, min(tl * ORBG_WAVE + lane, slen - 1));
            const uint64_t vmask = low_lanes(lim - t * ORBG_WAVE);
            const S syn = entry_syndrome<S>(L, cur);
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
            if (step(entA, entB)) break;
            if (step(entB, entA)) break;
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
        write_codeword<NK, S>(ybit, L, win_lo, win_hi, make_buf(cw_row, row_ok ? (uint32_t)n : 0u), NoOffs{});
        write_result(q_out, ab_out, found ? q : budget, !found);
    }
    __syncthreads();
}

template <int NKMAX, typename S, bool MIXED, int G, bool ONELINE>
__global__ void __launch_bounds__(G * ORBG_WAVE)
heavy_kernel(CodeTable codes, const uint8_t* __restrict__ block_code, const int64_t* __restrict__ row_off,
             const float* __restrict__ llr, uint32_t budget, uint32_t split_steps,
             uint8_t* __restrict__ cw, uint64_t* __restrict__ queries, uint8_t* __restrict__ abandoned,
             unsigned long long* __restrict__ ctrs, const int64_t* __restrict__ heavy, int64_t row_limit)
{
    __shared__ S s_cols[ORBG_WAVE * NKMAX];
    __shared__ BlockLds<S> L;
    __shared__ uint32_t best;
    __shared__ int s_j0;
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
        int64_t row = MIXED ? uniform_i64(row_off[b]) : b * c.n;
        // as in the light pass: a row outside the buffers is read as zeros, its stores dropped
        const bool row_ok = !MIXED || (row >= 0 && row <= row_limit - c.n);
        row = row_ok ? row : 0;
        if (c.nk == 1 || NKMAX == 1) {
            heavy_block<1, S, G, ONELINE>(c, llr + row, s_cols, L, &best, &s_j0, budget, split_steps, cw + row, queries + b,
                                 abandoned + b, row_ok);
        } else if (c.nk == 2 || NKMAX == 2) {
            constexpr int K2 = NKMAX >= 2 ? 2 : 1;
            heavy_block<K2, S, G, ONELINE>(c, llr + row, s_cols, L, &best, &s_j0, budget, split_steps, cw + row, queries + b,
                                  abandoned + b, row_ok);
        } else if (c.nk == 4 || NKMAX == 4) {
            constexpr int K4 = NKMAX >= 4 ? 4 : 1;
            heavy_block<K4, S, G, ONELINE>(c, llr + row, s_cols, L, &best, &s_j0, budget, split_steps, cw + row, queries + b,
                                  abandoned + b, row_ok);
        } else {
            heavy_block<NKMAX, S, G, ONELINE>(c, llr + row, s_cols, L, &best, &s_j0, budget, split_steps, cw + row, queries + b,
                                     abandoned + b, row_ok);
        }
    }
}

// Counters before a light pass: zero, but each slice counter past the slice's
// fixed first chunks (slice_start blocks).
static __global__ void reset_counters_kernel(unsigned long long* c, unsigned long long slice_start)
{
    for (int i = threadIdx.x; i < ORBG_CTR_WORDS; i += blockDim.x) c[i] = 0ull;
    __syncthreads();
    for (int i = threadIdx.x; i < ORBG_SLICES; i += blockDim.x) c[ORBG_CTR_SLICE(i)] = slice_start;
}

template <int NKMAX, bool ORDERED, typename S, bool MIXED, bool ONELINE>
static void launch_light(const DecodeArgs& a, int64_t wgs, int chunk, uint32_t split, hipStream_t stream)
{
    uint32_t ncols = 0;
    for (int i = 0; i < (MIXED ? a.codes.ncodes : 1); ++i) {
        const uint32_t e = a.codes.c[i].col_base + (uint32_t)a.codes.c[i].n;
        ncols = e > ncols ? e : ncols;
    }
    const size_t lds = (size_t)a.codes.rwords * sizeof(uint64_t) + ncols * sizeof(S);
    uint32_t fixed = 0;
    if (!a.p.naive) {
        // workgroups per slice resident from the start take fixed first chunks
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, light_kernel<NKMAX, ORDERED, S, MIXED, ONELINE>,
                                                         ORBG_WAVE, lds) != hipSuccess)
            per_cu = 0;
        const int64_t resident = (int64_t)per_cu * a.cus;
        fixed = (uint32_t)((resident < wgs ? resident : wgs) / ORBG_SLICES);
        reset_counters_kernel<<<1, 64, 0, stream>>>(a.ctrs, (unsigned long long)fixed * (unsigned long long)chunk);
    }
    light_kernel<NKMAX, ORDERED, S, MIXED, ONELINE><<<(unsigned)wgs, ORBG_WAVE, lds, stream>>>(
        a.codes, a.block_code, a.row_off, a.llr, a.nblocks, a.budget, split, a.order, a.cw, a.queries,
        a.abandoned, a.ctrs, a.heavy, chunk, a.j0, a.row_limit, a.ids, a.skip0 ? 1u : 0u, a.p.naive, fixed);
}

template <int NKMAX, typename S, bool MIXED, int G, bool ONELINE>
static void launch_heavy_g(const DecodeArgs& a, uint32_t split, hipStream_t stream)
{
    const int64_t wgs = (int64_t)a.cus * (a.p.heavy_wg_per_cu > 0 ? a.p.heavy_wg_per_cu : 2);
    heavy_kernel<NKMAX, S, MIXED, G, ONELINE><<<(unsigned)wgs, G * ORBG_WAVE, 0, stream>>>(
        a.codes, a.block_code, a.row_off, a.llr, a.budget, split, a.cw, a.queries, a.abandoned, a.ctrs, a.heavy,
        a.row_limit);
}

template <int NKMAX, bool ORDERED, typename S, bool MIXED, bool ONELINE = false>
static hipError_t launch_all(const DecodeArgs& a, hipStream_t stream)
{
    if (a.p.naive) {                                    // one one-wave workgroup per block
        if (a.nblocks > 0x7fffffffll) return hipErrorInvalidValue;
        launch_light<NKMAX, ORDERED, S, MIXED, ONELINE>(a, a.nblocks, 1, 0u, stream);
        return hipGetLastError();
    }
    int64_t wgs = a.nblocks;
    const int64_t cap = (int64_t)a.cus * (a.p.wg_per_cu > 0 ? a.p.wg_per_cu : 32);
    if (wgs > cap) wgs = cap;
    int chunk = a.p.chunk;
    if (chunk <= 0) {
        // about 4 chunks per wave: a counter increment is a round trip to L2,
        // so chunks stay as long as the balance at the end allows; a whole
        // number of screening groups when that is one or more (a chunk's last
        // group is not cut short)
        constexpr int K = ScreenDepth<NKMAX>::value;
        int64_t c = a.nblocks / (wgs * 4);
        c = c < 1 ? 1 : (c > 64 ? 64 : c);
        chunk = (int)(c >= K ? c - c % K : c);
    }
    chunk = chunk > 64 ? 64 : chunk;                    // a chunk's blocks fit one 64-bit mask
    const uint32_t split = (a.heavy != nullptr && a.p.split_steps > 0) ? (uint32_t)a.p.split_steps : 0u;
    launch_light<NKMAX, ORDERED, S, MIXED, ONELINE>(a, wgs, chunk, split, stream);
    if (split && !a.list_only) {
        if (a.p.heavy_waves >= 16) launch_heavy_g<NKMAX, S, MIXED, 16, ONELINE>(a, split, stream);
        else if (a.p.heavy_waves >= 8) launch_heavy_g<NKMAX, S, MIXED, 8, ONELINE>(a, split, stream);
        else launch_heavy_g<NKMAX, S, MIXED, 4, ONELINE>(a, split, stream);
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

template <int NKMAX>
static hipError_t launch_oneline(const DecodeArgs& a, bool s32, hipStream_t stream)
{
    if (s32) return launch_all<NKMAX, false, uint32_t, false, true>(a, stream);
    return launch_all<NKMAX, false, uint64_t, false, true>(a, stream);
}

// Launch of every decode mode with NKMAX keys per lane (instantiated once per
// NKMAX, each in its own translation unit).
template <int NKMAX>
hipError_t launch_decode_nk(const DecodeArgs& a, bool s32, hipStream_t stream)
{
    if (a.oneline) return launch_oneline<NKMAX>(a, s32, stream);
    if (a.mixed) {
        if constexpr (NKMAX <= 4) return launch_nk<NKMAX, true>(a, s32, stream);
        return hipErrorInvalidValue;                    // mixed launches take n <= 256
    }
    return launch_nk<NKMAX, false>(a, s32, stream);
}

}  // namespace orbg
