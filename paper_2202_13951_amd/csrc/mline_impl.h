// Full (m-line) ORBGRAND decode kernel for gfx950 (Sec. III-D; fit of Sec. III-E):
// the kernel template, compiled once per largest segment count by
// mline_m1.hip .. mline_m4.hip (the subset-count table and the launch dispatch
// are in mline.hip).
//
// Per block, one wave:
//   1. the LLR row (n <= 512: up to eight elements per lane), hard decision and
//      base syndrome s0 (Sec. III-A); s0 == 0 is query 1;
//   2. the full reliability order: keys (IEEE bits of |LLR|) << 32 | index sorted
//      ascending by a register bitonic network; h_r = column of rank r, pi_r its
//      received index and L_r its magnitude go to LDS;
//   3. the piecewise-linear fit (anchor points from ranks 1 and floor(n/2),
//      each added anchor at the largest vertical gap to the chord of its two
//      neighbours, the gaps of all candidate ranks computed one per lane) and
//      the quantization of eqs. (Q) and (quant), every FP32 operation rounded to
//      nearest in the written order; optionally J_{i-1} rounded to a multiple of
//      beta_i (the J/beta variant);
//   4. the query order of eq. (cartP): reliability weights W ascending; inside
//      one W the splitting patterns (W_1, ..., W_m) in the nested-loop order of
//      the integer splitting algorithm, each W_i among the partial weights its
//      segment can take (the collection step); inside one split the Cartesian
//      product of the partial sets, segment 1 outermost, each partial set by
//      partial Hamming weight, then Landslide (= lexicographic) order.  Below
//      weight 1024 the splits and the next weight come from per-block bitmaps
//      of the weights each segment and each suffix of segments can reach;
//      above, one pass per weight scans the candidates 64 at a time.  Each
//      split joins a queue in LDS, and the queued patterns are tested up to 64
//      at a time across splits and
//      weights: lane l takes the l-th untested pattern, finds its split and
//      unranks it (mixed radix over the segments, then the Hamming weight, then
//      a lexicographic subset of the segment's ranks with the given sum) with a
//      table of subset counts; a ballot of syndrome == 0 gives the first member
//      in order;
//   5. codeword, queries, abandon flag; optionally the block's segment count.
//
// Exactness limits (checked by the host): n <= 512, n - k <= 64, m <= 4,
// budget <= 5 x 10^6.  Every rank but rank 1 weighs at least 1 and rank 1 at
// least 0, so dropping flips from a pattern gives one that comes earlier (less
// weight, or the same weight, split and other segments with fewer flips in
// segment 1, which the order puts first).  A pattern with f flips therefore
// has the 2^f - 1 patterns made of proper subsets of its flips before it: no
// query within 5 x 10^6 < 2^23 - 1 has more than 22 flips.  Nor does one reach
// a relative logistic weight (sum of positions inside a segment) of 4096 or
// more: with w flips that needs w floor(4095 / w) < 4096 <= the segment's
// largest sum, so the segment is longer than K = floor(4095 / w), and the
// C(K, w) patterns that replace those w flips by w positions out of 1..K
// (w <= 22: at least C(186, 22), and C(455, 9) for the fewest flips a segment
// of 512 ranks needs) all weigh less.  The count table covers w <= 22 and
// relative weights below 4096; the order restricted to them agrees with the
// full order on its first 5 x 10^6 patterns, and every division below has
// operands under 2^32 (4095 times a slope of at most 2^20).
#pragma once
#include "orbg_device.h"
#include "orbg_internal.h"
#include "orbg_mline.h"

namespace orbg {

namespace {

constexpr int WL = ORBG_ML_WMAX;          // partial Hamming weights 0..22
constexpr int SL = ORBG_ML_SMAX;          // partial logistic weights 0..4095
constexpr int64_t NONE = INT64_MAX;

__device__ __forceinline__ uint32_t uni32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Subset counts: number of w-subsets of {1..len} with sum s, saturated.
__device__ __forceinline__ uint32_t subset_count(const uint32_t* __restrict__ tbl, int64_t len, int64_t w, int64_t s)
{
    if (len < 0 || len > ORBG_ML_LMAX || w < 0 || w > WL || s < 0 || s >= SL) return 0u;
    return tbl[((size_t)len * (WL + 1) + (size_t)w) * SL + (size_t)s];
}

__device__ __forceinline__ int64_t lw_min(int64_t w) { return w * (w + 1) / 2; }

// One segment of the model: offset J_{i-1}, slope beta_i, first rank - 1,
// length, and rcp = floor((2^32 - 1) / beta_i) for division by beta_i.
struct Seg {
    int64_t J, B;
    int off, len;
    uint32_t rcp;
};

__device__ __forceinline__ int wcap(const Seg& g) { return g.len < WL ? g.len : WL; }

// d / beta and d % beta for d < 2^32 by one high multiply: the error of rcp
// against 2^32 / beta is at most 1, so floor(d rcp / 2^32) is the quotient or
// one less, and one remainder test corrects it.
__device__ __forceinline__ uint32_t seg_div(const Seg& g, uint32_t d, uint32_t& rem)
{
    const uint32_t b = (uint32_t)g.B;
    uint32_t q = __umulhi(d, g.rcp);
    uint32_t r = d - q * b;
    if (r >= b) {
        ++q;
        r -= b;
    }
    rem = r;
    return q;
}

// The partial weights of w flips in a segment run from lo_w = w J + beta
// w(w+1)/2 to hi_w = w J + beta min(w len - w(w-1)/2, 4095) in steps of beta
// (relative weight, the sum of the positions inside the segment, from
// w(w+1)/2 up, capped below 4096).  lo_w grows strictly with w (by J +
// beta (w+1) >= beta w > 0, as J >= -beta), so a scan over w for a weight x
// stops at the first lo_w above x.  hi_w - lo_w < 4095 beta <= 2^32 - 2^20
// (beta <= 2^20): offsets inside one range are 32-bit.  SegScan steps through
// w = 1, 2, ... and keeps lo_w, hi_w.
struct SegScan {
    int64_t wJ, bs, lo, hi;
    int w, lmax;
    __device__ __forceinline__ explicit SegScan() : wJ(0), bs(0), lo(0), hi(0), w(0), lmax(0) {}
    __device__ __forceinline__ void next(const Seg& g)
    {
        ++w;
        wJ += g.J;
        bs += g.B * w;                         // beta w(w+1)/2
        lo = wJ + bs;
        lmax += g.len - (w - 1);               // w len - w(w-1)/2
        const int top = lmax < SL - 1 ? lmax : SL - 1;
        hi = wJ + (int64_t)((uint32_t)g.B * (uint32_t)top);
    }
};

// Number of partial patterns (at most 22 flips) of the segment with partial
// weight x; the empty one has weight 0.
__device__ uint64_t seg_count(const uint32_t* __restrict__ tbl, const Seg& g, int64_t x)
{
    uint64_t c = x == 0 ? 1u : 0u;
    const int wc = wcap(g);
    SegScan sc;
    for (int w = 1; w <= wc; ++w) {
        sc.next(g);
        if (sc.lo > x) break;
        if (x <= sc.hi) {
            uint32_t rem;
            const uint32_t q = seg_div(g, (uint32_t)(x - sc.lo), rem);
            if (rem == 0) c += subset_count(tbl, g.len, w, lw_min(w) + q);
        }
    }
    return c;
}

// Smallest partial weight >= x the segment can take (NONE if none).  In range
// w, the smallest weight >= x is lo_w + ceil((x - lo_w) / beta) beta, with
// x - lo_w + beta - 1 < 2^32.
__device__ int64_t seg_next(const Seg& g, int64_t x)
{
    if (x <= 0) return 0;
    int64_t best = NONE;
    const int wc = wcap(g);
    SegScan sc;
    for (int w = 1; w <= wc; ++w) {
        sc.next(g);
        if (sc.lo >= x) {
            // larger w only give more
            best = sc.lo < best ? sc.lo : best;
            break;
        }
        if (x <= sc.hi) {
            uint32_t rem;
            const uint32_t q = seg_div(g, (uint32_t)(x - sc.lo) + (uint32_t)g.B - 1u, rem);
            const int64_t c = sc.lo + (int64_t)q * g.B;
            best = c < best ? c : best;
        }
    }
    return best;
}

// Both of the above at once for y >= 0: the count at y and the smallest weight
// above y (the smallest in range w above y is lo_w + (floor((y - lo_w) / beta)
// + 1) beta, if that is <= hi_w).
__device__ void seg_count_next(const uint32_t* __restrict__ tbl, const Seg& g, int64_t y, uint64_t& cnt,
                               int64_t& nxt)
{
    uint64_t c = y == 0 ? 1u : 0u;
    int64_t best = NONE;
    const int wc = wcap(g);
    SegScan sc;
    for (int w = 1; w <= wc; ++w) {
        sc.next(g);
        if (sc.lo > y) {
            best = sc.lo < best ? sc.lo : best;
            break;
        }
        if (y <= sc.hi) {
            uint32_t rem;
            const uint32_t q = seg_div(g, (uint32_t)(y - sc.lo), rem);
            if (rem == 0) c += subset_count(tbl, g.len, w, lw_min(w) + q);
            const int64_t up = sc.lo + (int64_t)(q + 1u) * g.B;
            if (up <= sc.hi) best = up < best ? up : best;
        }
    }
    cnt = c;
    nxt = best;
}

// Can the segment take partial weight x (some partial Hamming weight <= 22)?
__device__ __forceinline__ bool seg_member(const Seg& g, int64_t x)
{
    if (x == 0) return true;
    const int wc = wcap(g);
    SegScan sc;
    for (int w = 1; w <= wc; ++w) {
        sc.next(g);
        if (sc.lo > x) break;
        if (x <= sc.hi) {
            uint32_t rem;
            (void)seg_div(g, (uint32_t)(x - sc.lo), rem);
            if (rem == 0) return true;
        }
    }
    return false;
}

// Minimum of an i64 over the wave, wave-uniform (all lanes active): quad
// swaps, half-row and row mirrors inside each 16-lane row, then the four rows.
__device__ __forceinline__ int64_t dpp_min_step(int64_t v, int ctrl_sel)
{
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)((uint64_t)v >> 32);
    uint32_t l2, h2;
    switch (ctrl_sel) {
    case 0:
        l2 = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, 0xB1, 0xF, 0xF, false);
        h2 = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, 0xB1, 0xF, 0xF, false);
        break;
    case 1:
        l2 = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, 0x4E, 0xF, 0xF, false);
        h2 = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, 0x4E, 0xF, 0xF, false);
        break;
    case 2:
        l2 = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, 0x141, 0xF, 0xF, false);
        h2 = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, 0x141, 0xF, 0xF, false);
        break;
    default:
        l2 = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, 0x140, 0xF, 0xF, false);
        h2 = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, 0x140, 0xF, 0xF, false);
        break;
    }
    const int64_t o = (int64_t)(((uint64_t)h2 << 32) | l2);
    return o < v ? o : v;
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t v)
{
    v = dpp_min_step(v, 0);
    v = dpp_min_step(v, 1);
    v = dpp_min_step(v, 2);
    v = dpp_min_step(v, 3);
    const uint64_t u = (uint64_t)v;
    int64_t m = NONE;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t l = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 16 * r);
        const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 16 * r);
        const int64_t x = (int64_t)(((uint64_t)h << 32) | l);
        m = x < m ? x : m;
    }
    return m;
}

// seg_next for a wave-uniform x (all lanes active), one Hamming weight per
// lane: every w's smallest weight >= x, then their minimum.
__device__ int64_t seg_next_wave(const Seg& g, int64_t x)
{
    if (x <= 0) return 0;
    const int w = lane_id() + 1;
    int64_t c = NONE;
    if (w <= wcap(g)) {
        const int64_t wJ = (int64_t)w * g.J;
        const int64_t lo = wJ + g.B * lw_min(w);
        if (lo >= x) {
            c = lo;
        } else {
            const int lm = w * g.len - w * (w - 1) / 2;
            const int top = lm < SL - 1 ? lm : SL - 1;
            const int64_t hi = wJ + (int64_t)((uint32_t)g.B * (uint32_t)top);
            if (x <= hi) {
                uint32_t rem;
                const uint32_t q = seg_div(g, (uint32_t)(x - lo) + (uint32_t)g.B - 1u, rem);
                c = lo + (int64_t)q * g.B;
            }
        }
    }
    return wave_min_i64(c);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}


// A split waiting to be tested (LDS ring of ORBG_ML_QCAP entries): its partial
// weights, partial-set sizes (saturated at 2^32 - 1, exact for product indices
// below the budget), the first product element not yet tested and the number of
// elements to test (the product size, cut at the budget).
struct QEntry {
    int64_t a[ORBG_ML_MSEG];
    uint32_t cnt[ORBG_ML_MSEG];
    uint32_t first, total;
};

// Weights below X0 are walked from per-block bitmaps (the walk of a block
// rarely passes weight 255, almost never 1023): R_i, the partial weights
// segment i can take; S_i = R_i + R_{i+1} + ... + R_{m-1} (Minkowski sums), the
// totals of segments i..m-1 that some split reaches; rS_i, S_i reflected (bit
// j for weight X0 - 1 - j); and the partial-set sizes of the weights below CX,
// saturated at 2^32 - 1 (larger ones are counted when needed).  Words are
// built as the walk's weight reaches them.
constexpr int XW = 16;
constexpr int X0 = 64 * XW;
constexpr int CX = 256;

struct MlMaps {
    uint64_t R[ORBG_ML_MSEG][XW];
    uint64_t S[ORBG_ML_MSEG][XW];
    uint64_t rS[ORBG_ML_MSEG][XW];
    uint32_t cnt[ORBG_ML_MSEG][CX];
};

template <int M>
struct Walk {
    Seg seg[M];
    int64_t a[M];           // current split
    uint32_t cnt[M];        // partial-set sizes of the split, saturated at 2^32 - 1
    uint64_t qbase;         // patterns tested
    uint32_t pending;       // patterns queued, not yet tested
    uint32_t want;          // queued patterns that start a test: 2, doubling to 64
    int qhead, live;        // ring position and number of queued splits
    uint32_t budget;
    uint64_t s0;
    const uint32_t* tbl;
    const uint64_t* h;      // LDS: column of each rank
    uint16_t* win;          // LDS: the winner's ranks
    QEntry* Q;              // LDS: queued splits
    MlMaps* mp;             // LDS: bitmaps and partial-set sizes below X0
    int built;              // bitmap words built
    int nwin;
    bool stop, found;
    bool dry;               // enumerate without queueing (the step past X0)
    uint32_t q;
};

// Lexicographic unranking of a w-subset of {1..len} with sum s: index u (0-based)
// among those subsets in ascending order of (v_1, v_2, ...).  emit(v) per
// element.  Each element but the last two scans its candidates c upward: the
// rw elements after v_k = c come from {c+1..len} with sum s - c, i.e. (shifted
// by c) from {1..len-c} with sum s - c - rw c.
// The last two have closed forms: the pairs from {prev+1..len} with sum s are
// (c, s - c) for c from max(prev + 1, s - len) to floor((s - 1) / 2), one for
// each c, and a last element alone is s.
template <typename F>
__device__ __forceinline__ void unrank_subset(const uint32_t* __restrict__ tbl, int len, int w, int64_t s, uint64_t u,
                                              F&& emit)
{
    int prev = 0;
    for (int k = 1; k <= w; ++k) {
        const int rw = w - k;
        int c;
        if (rw == 0) {
            c = (int)s;
        } else if (rw == 1) {
            const int64_t first = (int64_t)prev + 1 > s - len ? (int64_t)prev + 1 : s - len;
            c = (int)(first + (int64_t)u);
            u = 0;
        } else {
            c = prev + 1;
            for (; c <= len; ++c) {
                const uint64_t n = subset_count(tbl, len - c, rw, s - c - (int64_t)rw * c);
                if (u < n) break;
                u -= n;
            }
            if (c > len) c = len;         // exact counts always stop the scan before
        }
        emit(c);
        s -= c;
        prev = c;
    }
}

// Element u of the partial set of segment g for partial weight x: Hamming
// weight ascending (the empty pattern first), lexicographic inside.
template <typename F>
__device__ __forceinline__ void unrank_partial(const uint32_t* __restrict__ tbl, const Seg& g, int64_t x, uint64_t u,
                                               F&& emit)
{
    if (x == 0) {
        if (u == 0) return;                   // the empty partial pattern
        u -= 1;
    }
    const int wc = wcap(g);
    SegScan sc;
    for (int w = 1; w <= wc; ++w) {
        sc.next(g);
        if (sc.lo > x) break;
        if (x > sc.hi) continue;
        uint32_t rem;
        const uint32_t q = seg_div(g, (uint32_t)(x - sc.lo), rem);
        if (rem != 0) continue;
        const int64_t wp = lw_min(w) + q;
        const uint64_t n = subset_count(tbl, g.len, w, wp);
        if (u < n) {
            unrank_subset(tbl, g.len, w, wp, u, [&](int v) { emit(g.off + v); });
            return;
        }
        u -= n;
    }
}

// Product element u of a split (partial weights a, partial-set sizes cnt),
// segment 1 outermost.
template <int M, typename F>
__device__ __forceinline__ void unrank_product(const Seg (&seg)[M], const uint32_t* tbl, const int64_t (&a)[M],
                                               const uint32_t (&cnt)[M], uint32_t u, F&& emit)
{
    // u < 2^23: a radix above u leaves the digit u and quotient 0
    uint32_t t[M];
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        if (i == 0 || cnt[i] > u) {
            t[i] = u;
            u = 0;
        } else {
            t[i] = u % cnt[i];
            u = u / cnt[i];
        }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) unrank_partial(tbl, seg[i], a[i], t[i], emit);
}

__device__ __forceinline__ uint32_t sat32(uint64_t v) { return v < 0xffffffffull ? (uint32_t)v : 0xffffffffu; }

// Tests queued patterns up to 64 at a time in queue order while at least
// `want` are queued (all of them when `final`): lane l takes the l-th untested
// pattern, finds its split by the running sum of the queued counts and
// unranks it; a ballot gives the first member.  `want` starts at 2 (a block
// that decodes early is tested before much of the order is walked) and doubles
// to 64 per step.
template <int M>
__device__ __forceinline__ void flush(Walk<M>& c, bool final)
{
    const int lane = lane_id();
    wave_lds_sync();                          // queue entries written by lane 0
    while (!c.found && c.pending > 0 && (final || c.pending >= c.want)) {
        const uint32_t chunk = c.pending < (uint32_t)ORBG_WAVE ? c.pending : (uint32_t)ORBG_WAVE;
        c.want = c.want < (uint32_t)ORBG_WAVE ? 2 * c.want : (uint32_t)ORBG_WAVE;
        const bool act = (uint32_t)lane < chunk;
        bool got = false;
        int e = c.qhead;
        uint32_t idx = 0, acc = 0;
        for (int k = 0; k < c.live && acc < chunk; ++k) {
            const int sl = (c.qhead + k) % ORBG_ML_QCAP;
            const uint32_t rem = c.Q[sl].total - c.Q[sl].first;
            if (!got && (uint32_t)lane < acc + rem) {
                got = true;
                e = sl;
                idx = c.Q[sl].first + ((uint32_t)lane - acc);
            }
            acc += rem;
        }
        int64_t a[M];
        uint32_t cn[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            a[i] = act ? c.Q[e].a[i] : 0;
            cn[i] = act ? c.Q[e].cnt[i] : 1u;
        }
        uint64_t s = c.s0;
        if (act) unrank_product(c.seg, c.tbl, a, cn, idx, [&](int r) { s ^= c.h[r]; });
        const uint64_t hits = ballot(act && s == 0);
        if (hits != 0) {
            const int wl = __builtin_ctzll(hits);
            c.q = (uint32_t)(c.qbase + (uint64_t)wl + 1);
            c.found = true;
            c.stop = true;
            if (lane == wl) {
                int nw = 0;
                unrank_product(c.seg, c.tbl, a, cn, idx, [&](int r) {
                    if (nw < ORBG_ML_WINCAP) c.win[nw++] = (uint16_t)r;
                });
                c.win[ORBG_ML_WINCAP] = (uint16_t)nw;
            }
            wave_lds_sync();
            c.nwin = (int)uni32(c.win[ORBG_ML_WINCAP]);
            return;
        }
        // the chunk's patterns are tested: drop whole splits, advance the last one
        c.qbase += chunk;
        c.pending -= chunk;
        uint32_t left = chunk;
        while (left > 0) {
            const int sl = c.qhead;
            const uint32_t rem = uni32(c.Q[sl].total - c.Q[sl].first);
            if (rem <= left) {
                left -= rem;
                c.qhead = (c.qhead + 1) % ORBG_ML_QCAP;
                --c.live;
            } else {
                if (lane == 0) c.Q[sl].first += left;
                left = 0;
            }
        }
        wave_lds_sync();
    }
}

// Queues the current split (its product cut at the budget) and tests whole
// steps of 64 queued patterns; at the budget, tests the rest and stops.
template <int M>
__device__ __forceinline__ void push_split(Walk<M>& c)
{
    // product of the partial-set sizes (each below 2^32), capped at 2^32, which
    // is above any budget
    uint64_t count = 1;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        count *= c.cnt[i];
        count = count < (1ull << 32) ? count : (1ull << 32);
    }
    const uint64_t room = (uint64_t)c.budget - c.qbase - c.pending;        // > 0 while the walk runs
    const uint32_t tot = (uint32_t)(count < room ? count : room);
    const int slot = (c.qhead + c.live) % ORBG_ML_QCAP;                     // live < 64 here
    if (lane_id() == 0) {
        QEntry& q = c.Q[slot];
#pragma unroll
        for (int i = 0; i < ORBG_ML_MSEG; ++i) {
            q.a[i] = i < M ? c.a[i < M ? i : 0] : 0;
            q.cnt[i] = i < M ? c.cnt[i < M ? i : 0] : 1u;
        }
        q.first = 0;
        q.total = tot;
    }
    // (the entry is read in flush, which starts with an LDS sync)
    ++c.live;
    c.pending += tot;
    // the only call of flush (one inlined copy of the unranking per kernel)
    const bool fin = c.qbase + c.pending >= (uint64_t)c.budget;
    if (fin || c.pending >= c.want) flush<M>(c, fin);
    if (fin) c.stop = true;
}

// One pass over the splits of `rest` among segments I..M-1, in the nested-loop
// order of the splitting algorithm, queueing each; returns the smallest total
// weight of those segments above `rest` (NONE if none, or once the walk
// stops), which is where the walk goes next.  With W_I = a <= rest that total
// is a + (the same for segments I+1.. above rest - a); a value of segment I
// above rest stands alone (the later segments add 0), the smallest being its
// next value above rest.  Every level takes 64 candidate values of W_I at a
// time (lane l takes base + l; a ballot keeps the values the segment can take
// -- at the last two segments, the splits -- taken in ascending order), an
// empty stretch skipped to segment I's next value.
template <int I, int M>
__device__ __forceinline__ int64_t walk_level(Walk<M>& c, int64_t rest)
{
    const int64_t need = rest + 1;
    int64_t best = seg_next_wave(c.seg[I], need);
    if constexpr (I == M - 2) {
        const int lane = lane_id();
        for (int64_t base = 0; base <= rest;) {
            // per lane: candidate W_I = a, the partial-set sizes of (a, rest - a)
            // and the next total above rest through a
            const int64_t a = base + lane;
            const bool m0 = a <= rest && seg_member(c.seg[I], a);
            uint64_t n0 = 0, n1 = 0;
            int64_t cand = NONE;
            if (m0) {
                int64_t r;
                seg_count_next(c.tbl, c.seg[I + 1], rest - a, n1, r);
                if (n1 != 0) n0 = seg_count(c.tbl, c.seg[I], a);
                if (r != NONE) cand = a + r;
            }
            const int64_t mn = wave_min_i64(cand);
            best = mn < best ? mn : best;
            for (uint64_t bal = ballot(n1 != 0); bal != 0 && !c.stop; bal &= bal - 1) {
                const int l = __builtin_ctzll(bal);
                const int64_t av = base + (int64_t)l;
                c.a[I] = av;
                c.cnt[I] = sat32(readlane_u64(n0, l));
                c.a[I + 1] = rest - av;
                c.cnt[I + 1] = sat32(readlane_u64(n1, l));
                if (!c.dry) push_split<M>(c);
            }
            if (c.stop) return NONE;
            base = seg_next_wave(c.seg[I], base + ORBG_WAVE);
        }
    } else {
        // 64 candidate values of W_I per step: membership and partial-set size
        // per lane, then the members in ascending order
        const int lane = lane_id();
        for (int64_t base = 0; base <= rest;) {
            const int64_t a = base + lane;
            const uint64_t n0 = a <= rest ? seg_count(c.tbl, c.seg[I], a) : 0;
            for (uint64_t bal = ballot(n0 != 0); bal != 0; bal &= bal - 1) {
                const int l = __builtin_ctzll(bal);
                const int64_t av = base + (int64_t)l;
                c.a[I] = av;
                c.cnt[I] = sat32(readlane_u64(n0, l));
                const int64_t r = walk_level<I + 1, M>(c, rest - av);
                if (c.stop) return NONE;
                if (r != NONE && av + r < best) best = av + r;
            }
            base = seg_next_wave(c.seg[I], base + ORBG_WAVE);
        }
    }
    return best;
}

__device__ __forceinline__ uint64_t lds_u64(const uint64_t* p) { return uniform_u64(*p); }
__device__ __forceinline__ uint32_t lds_u32(const uint32_t* p) { return uni32(*p); }

__device__ __forceinline__ uint64_t bitrev64(uint64_t v)
{
    return ((uint64_t)__builtin_bitreverse32((uint32_t)v) << 32) | __builtin_bitreverse32((uint32_t)(v >> 32));
}

// OR of a u64 over the wave, wave-uniform (all lanes active).
__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#define ORBG_OR_STEP(ctrl)                                                                    \
    lo |= (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, ctrl, 0xF, 0xF, false);    \
    hi |= (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, ctrl, 0xF, 0xF, false);
    ORBG_OR_STEP(0xB1)      // quad_perm [1,0,3,2]
    ORBG_OR_STEP(0x4E)      // quad_perm [2,3,0,1]
    ORBG_OR_STEP(0x141)     // row_half_mirror
    ORBG_OR_STEP(0x140)     // row_mirror
#undef ORBG_OR_STEP
    const uint32_t l = __builtin_amdgcn_readlane(lo, 0) | __builtin_amdgcn_readlane(lo, 16) |
                       __builtin_amdgcn_readlane(lo, 32) | __builtin_amdgcn_readlane(lo, 48);
    const uint32_t h = __builtin_amdgcn_readlane(hi, 0) | __builtin_amdgcn_readlane(hi, 16) |
                       __builtin_amdgcn_readlane(hi, 32) | __builtin_amdgcn_readlane(hi, 48);
    return ((uint64_t)h << 32) | l;
}

// seg_count for a wave-uniform x (all lanes active), one Hamming weight per
// lane, saturated at 2^32 - 1.
__device__ uint32_t seg_count_wave(const uint32_t* __restrict__ tbl, const Seg& g, int64_t x)
{
    const int w = lane_id() + 1;
    uint64_t t = 0;
    if (w <= wcap(g)) {
        const int64_t wJ = (int64_t)w * g.J;
        const int64_t lo = wJ + g.B * lw_min(w);
        const int lm = w * g.len - w * (w - 1) / 2;
        const int top = lm < SL - 1 ? lm : SL - 1;
        const int64_t hi = wJ + (int64_t)((uint32_t)g.B * (uint32_t)top);
        if (lo <= x && x <= hi) {
            uint32_t rem;
            const uint32_t q = seg_div(g, (uint32_t)(x - lo), rem);
            if (rem == 0) t = subset_count(tbl, g.len, w, lw_min(w) + q);
        }
    }
    uint32_t lo = (uint32_t)t, hi = (uint32_t)(t >> 32);
#define ORBG_ADD_STEP(ctrl)                                                                          \
    {                                                                                                \
        const uint32_t l2 = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, ctrl, 0xF, 0xF, false); \
        const uint32_t h2 = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, ctrl, 0xF, 0xF, false); \
        const uint64_t v = (((uint64_t)hi << 32) | lo) + (((uint64_t)h2 << 32) | l2);                  \
        lo = (uint32_t)v;                                                                            \
        hi = (uint32_t)(v >> 32);                                                                    \
    }
    // every lane ends with the sum over its 16-lane row (each step pairs lanes
    // holding sums over disjoint sets)
    ORBG_ADD_STEP(0xB1)      // quad_perm [1,0,3,2]
    ORBG_ADD_STEP(0x4E)      // quad_perm [2,3,0,1]
    ORBG_ADD_STEP(0x141)     // row_half_mirror
    ORBG_ADD_STEP(0x140)     // row_mirror
#undef ORBG_ADD_STEP
    uint64_t sum = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        sum += ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, 16 * r) << 32) |
               (uint32_t)__builtin_amdgcn_readlane((int)lo, 16 * r);
    if (x == 0) sum += 1;
    return sum > 0xffffffffull ? 0xffffffffu : (uint32_t)sum;
}

// Partial-set size of weight x < X0 of segment i: the cached one below CX.
template <int M>
__device__ __forceinline__ uint32_t map_count(Walk<M>& c, int i, int x)
{
    if (x < CX) return lds_u32(&c.mp->cnt[i][x]);
    return seg_count_wave(c.tbl, c.seg[i], x);
}

// Builds word k of every map (weights 64k .. 64k + 63): partial-set sizes and
// R_i, one weight per lane; then S_i from the last segment back: word k of
// S_i is the OR over a in R_i (a < 64 (k + 1)) of word k of S_{i+1} shifted
// up by a, 64 values of a per pass (lane l: a = 64 p + l, shift l of words
// k - p and k - p - 1); rS_i gets the word reflected.
template <int M>
__device__ __forceinline__ void build_word(Walk<M>& c, int k)
{
    const int lane = lane_id();
    MlMaps& mp = *c.mp;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int x = 64 * k + lane;
        bool mem;
        if (x < CX) {
            const uint64_t n = seg_count(c.tbl, c.seg[i], x);
            mp.cnt[i][x] = n > 0xffffffffull ? 0xffffffffu : (uint32_t)n;
            mem = n != 0;
        } else {
            mem = seg_member(c.seg[i], x);
        }
        const uint64_t r = ballot(mem);
        if (lane == 0) mp.R[i][k] = r;
        if (i == M - 1 && lane == 0) {
            mp.S[i][k] = r;
            mp.rS[i][XW - 1 - k] = bitrev64(r);
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int i = M - 2; i >= 0; --i) {
        uint64_t acc = 0;
        for (int p = 0; p <= k; ++p) {
            const uint64_t member = lds_u64(&mp.R[i][p]);
            const uint64_t hi = lds_u64(&mp.S[i + 1][k - p]);
            const uint64_t lo = k - p - 1 >= 0 ? lds_u64(&mp.S[i + 1][k - p - 1]) : 0ull;
            const uint64_t w = lane == 0 ? hi : (hi << lane) | (lo >> (64 - lane));
            acc |= ((member >> lane) & 1ull) ? w : 0ull;
        }
        const uint64_t sk = wave_or_u64(acc);
        if (lane == 0) {
            mp.S[i][k] = sk;
            mp.rS[i][XW - 1 - k] = bitrev64(sk);
        }
        wave_lds_sync();
    }
}

// Queues every split of `rest` (< 64 built words) over segments I..M-1 in the
// nested-loop order: the values a <= rest of R_I with rest - a in S_{I+1}, as
// the AND of R_I with rS_{I+1} shifted down by X0 - 1 - rest (bit a of the
// shifted map is bit rest - a of S_{I+1}; a > rest falls past the map).
template <int I, int M>
__device__ __forceinline__ void enum_splits(Walk<M>& c, int rest)
{
    MlMaps& mp = *c.mp;
    const int d = X0 - 1 - rest, q = d >> 6, r = d & 63;
    for (int j = 0; j <= (rest >> 6); ++j) {
        const uint64_t lo = j + q < XW ? lds_u64(&mp.rS[I + 1][j + q]) : 0ull;
        const uint64_t hi = j + q + 1 < XW ? lds_u64(&mp.rS[I + 1][j + q + 1]) : 0ull;
        const uint64_t sh = r == 0 ? lo : (lo >> r) | (hi << (64 - r));
        uint64_t bits = lds_u64(&mp.R[I][j]) & sh;
        while (bits != 0) {
            const int a = 64 * j + __builtin_ctzll(bits);
            bits &= bits - 1;
            c.a[I] = a;
            c.cnt[I] = map_count(c, I, a);
            if constexpr (I == M - 2) {
                c.a[I + 1] = rest - a;
                c.cnt[I + 1] = map_count(c, I + 1, rest - a);
                push_split<M>(c);
            } else {
                enum_splits<I + 1, M>(c, rest - a);
            }
            if (c.stop) return;
        }
    }
}

// Smallest total weight above W from S_0, building words as needed; -1 when
// there is none below X0.
template <int M>
__device__ __forceinline__ int64_t next_total_map(Walk<M>& c, int64_t W)
{
    for (int64_t t = W + 1; t < X0;) {
        const int k = (int)(t >> 6);
        if (k >= c.built) {
            build_word<M>(c, k);
            c.built = k + 1;
        }
        const uint64_t bits = lds_u64(&c.mp->S[0][k]) & (~0ull << (t & 63));
        if (bits != 0) return 64 * k + __builtin_ctzll(bits);
        t = 64 * (int64_t)(k + 1);
    }
    return -1;
}

// Reliability weights in increasing order, each one's splits queued and tested.
// No weight left (NONE) is only possible once the query limit is reached (the
// limit is at most 2^n, and the restricted order holds min(2^n, the budget)
// patterns at least), so the queue has been tested by then.
template <int M>
__device__ __forceinline__ void walk(Walk<M>& c)
{
    // weights below X0 from the maps
    {
        MlMaps& mp = *c.mp;
        const int lane = lane_id();
        uint64_t* words = &mp.R[0][0];
        for (int i = lane; i < 3 * ORBG_ML_MSEG * XW; i += ORBG_WAVE) words[i] = 0ull;
        wave_lds_sync();
        build_word<M>(c, 0);
        c.built = 1;
    }
    int64_t W = 0;
    for (;;) {
        if constexpr (M == 1) {
            if ((lds_u64(&c.mp->R[0][W >> 6]) >> (W & 63)) & 1ull) {
                c.a[0] = W;
                c.cnt[0] = map_count(c, 0, (int)W);
                push_split<1>(c);
            }
        } else {
            enum_splits<0, M>(c, (int)W);
        }
        if (c.stop) return;
        const int64_t nx = next_total_map<M>(c, W);
        if (nx < 0) break;
        W = nx;
    }
    // the first weight at or above X0: one pass over the splits of X0 - 1
    // without queueing them (they were queued from the maps)
    int64_t nxt;
    if constexpr (M == 1) {
        nxt = seg_next_wave(c.seg[0], X0);
    } else {
        c.dry = true;
        nxt = walk_level<0, M>(c, X0 - 1);
        c.dry = false;
    }
    if (nxt == NONE) return;
    W = uni64(nxt);
    for (;;) {
        if constexpr (M == 1) {
            const uint64_t n = seg_count(c.tbl, c.seg[0], W);
            if (n != 0) {
                c.a[0] = W;
                c.cnt[0] = sat32(n);
                push_split<1>(c);
            }
            nxt = seg_next_wave(c.seg[0], W + 1);
        } else {
            nxt = walk_level<0, M>(c, W);
        }
        if (c.stop || nxt == NONE) return;
        W = uni64(nxt);
    }
}

__device__ __forceinline__ bool round_half_up(float x, int64_t& out)
{
    if (!__builtin_isfinite(x)) return false;
    float r = floorf(__fadd_rn(x, 0.5f));
    if (r > 1048576.0f) r = 1048576.0f;
    out = (int64_t)r;
    return true;
}

// LDS of one wave, for codes of at most LC ranks.
template <int LC>
struct MlLds {
    uint64_t h[LC + 1];                 // h[r] = column of rank r
    float L[LC + 1];                    // L[r] = |LLR| of rank r
    uint16_t pi[LC + 1];                // pi[r] = received index of rank r
    int anc[ORBG_ML_MSEG + 2];          // anchor ranks, ascending
    uint16_t win[ORBG_ML_WINCAP + 1];   // winner's ranks, then their count
    QEntry Q[ORBG_ML_QCAP];             // splits waiting to be tested
    MlMaps maps;                        // bitmaps of the walk below weight X0
};

struct Model {
    int m;
    int I[ORBG_ML_MSEG + 1];
    int64_t J[ORBG_ML_MSEG], B[ORBG_ML_MSEG];
};

__device__ __forceinline__ void model_basic(Model& md, int n)
{
    md.m = 1;
    md.I[0] = 0;
#pragma unroll
    for (int i = 1; i <= ORBG_ML_MSEG; ++i) md.I[i] = n;
#pragma unroll
    for (int i = 0; i < ORBG_ML_MSEG; ++i) { md.J[i] = 0; md.B[i] = 1; }
}

// Fit with at most mreq segments (L in LDS, ranks 1..n; h = n/2 <= 32 NK).
// Wave-uniform result.
template <int NK, typename Lds>
__device__ __forceinline__ Model fit_model(Lds& S, int n, int mreq, bool jdiv)
{
    const int lane = lane_id();
    Model md;
    model_basic(md, n);
    const int h = n / 2;
    if (h < 2) return md;
    if (lane == 0) { S.anc[0] = 1; S.anc[1] = h; }
    wave_lds_sync();
    int na = 2;
    for (int it = 1; it < mreq; ++it) {
        // candidate ranks j = l + 1 + 64 t of lane l (t < NK / 2: h <= 32 NK),
        // each strictly between two adjacent anchors: largest gap, smallest
        // rank on ties, as the max of (gap bits, 0xffff - j)
        auto gap_key = [&](int j) -> uint64_t {
            int a = 0, b = 0;
            for (int p = 0; p + 1 < na; ++p) {
                const int lo = S.anc[p], hi = S.anc[p + 1];
                if (j > lo && j < hi) { a = lo; b = hi; }
            }
            if (b == 0 || j > h) return 0ull;
            const float La = S.L[a], Lb = S.L[b];
            const float s = __fdiv_rn(__fsub_rn(Lb, La), (float)(b - a));
            const float t = __fmul_rn((float)(j - a), s);
            const float line = __fadd_rn(La, t);
            const float gap = fabsf(__fsub_rn(S.L[j], line));
            if (__builtin_isnan(gap)) return 0ull;
            return ((uint64_t)__float_as_uint(gap) << 32) | (uint64_t)(0xffff - j);
        };
        uint64_t key = gap_key(lane + 1);
#pragma unroll
        for (int t = 1; t < NK / 2; ++t) {
            const uint64_t k2 = gap_key(lane + 1 + t * ORBG_WAVE);
            key = k2 > key ? k2 : key;
        }
#pragma unroll
        for (int d = 1; d < ORBG_WAVE; d <<= 1) {
            const uint64_t o = __shfl_xor(key, d, ORBG_WAVE);
            key = o > key ? o : key;
        }
        key = (uint64_t)uni64((int64_t)key);
        if (key == 0ull) break;                                  // no rank left between anchors
        if ((uint32_t)(key >> 32) == 0u) break;                  // largest gap is 0
        const int bj = 0xffff - (int)(key & 0xffffffffull);
        if (lane == 0) {
            int p = na;
            while (p > 0 && S.anc[p - 1] > bj) { S.anc[p] = S.anc[p - 1]; --p; }
            S.anc[p] = bj;
        }
        wave_lds_sync();
        ++na;
    }
    const int m = na - 1;
    float d[ORBG_ML_MSEG], len[ORBG_ML_MSEG];
    float Q = 0.0f;
#pragma unroll
    for (int i = 0; i < ORBG_ML_MSEG; ++i) {
        if (i < m) {
            const int lo = S.anc[i], hi = S.anc[i + 1];
            d[i] = __fsub_rn(S.L[hi], S.L[lo]);
            len[i] = (float)(hi - lo);
            const float s = __fdiv_rn(d[i], len[i]);
            if (i == 0 || s < Q) Q = s;
        } else {
            d[i] = 0.0f;
            len[i] = 1.0f;
        }
    }
    if (!(Q > 0.0f) || !__builtin_isfinite(Q)) return md;
    Model r;
    r.m = m;
    r.I[0] = 0;
#pragma unroll
    for (int i = 1; i <= ORBG_ML_MSEG; ++i) r.I[i] = i < m ? S.anc[i] : n;
#pragma unroll
    for (int i = 0; i < ORBG_ML_MSEG; ++i) {
        r.J[i] = 0;
        r.B[i] = 1;
        if (i < m) {
            const float t = __fmul_rn(len[i], Q);
            if (!round_half_up(__fdiv_rn(d[i], t), r.B[i]) || r.B[i] < 1) return md;
        }
    }
    int64_t rb = 0;
    if (!round_half_up(__fdiv_rn(S.L[1], Q), rb)) return md;
    r.J[0] = rb - r.B[0];
#pragma unroll
    for (int i = 1; i < ORBG_ML_MSEG; ++i)
        if (i < m && !round_half_up(__fdiv_rn(S.L[S.anc[i]], Q), r.J[i])) return md;
    if (jdiv) {
#pragma unroll
        for (int i = 0; i < ORBG_ML_MSEG; ++i) {
            const int64_t num = 2 * r.J[i] + r.B[i], den = 2 * r.B[i];
            int64_t qq = num / den;
            if (num % den != 0 && num < 0) --qq;
            r.J[i] = qq * r.B[i];
        }
    }
    return r;
}

template <int M, typename Lds>
__device__ __forceinline__ void decode_walk(const Model& md, const uint32_t* tbl, Lds& S, uint64_t s0, uint32_t limit,
                            bool& found, uint32_t& q, int& nwin)
{
    Walk<M> c;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        c.seg[i].J = md.J[i];
        c.seg[i].B = md.B[i];
        c.seg[i].off = md.I[i];
        c.seg[i].len = md.I[i + 1] - md.I[i];
        c.seg[i].rcp = 0xffffffffu / (uint32_t)md.B[i];
    }
    c.qbase = 0;
    c.pending = 0;
    c.want = 2;
    c.qhead = 0;
    c.live = 0;
    c.Q = S.Q;
    c.budget = limit;
    c.s0 = s0;
    c.tbl = tbl;
    c.h = S.h;
    c.win = S.win;
    c.mp = &S.maps;
    c.built = 0;
    c.dry = false;
    c.nwin = 0;
    c.stop = false;
    c.found = false;
    c.q = limit;
    walk<M>(c);
    found = c.found;
    q = c.q;
    nwin = c.nwin;
}

// Five waves per SIMD for one or two keys per lane (the walk is latency-bound:
// measured 4% faster than the four the register count gives by itself, at a
// 20-byte spill for two keys); four keys keep the compiler's choice.  MM: the
// largest number of segments the launch's fits may use (a.mseg); only the
// walks up to MM are compiled into the kernel, which keeps the registers of a
// two-line decode free of the three- and four-line walks' state.
template <int NK, int MM>
__global__ void __launch_bounds__(ORBG_WAVE) __attribute__((amdgpu_waves_per_eu(NK <= 2 ? 5 : 1))) mline_kernel(MlineArgs a)
{
    __shared__ MlLds<NK * ORBG_WAVE> S;
    const int lane = lane_id();
    const int n = a.n;
    // rows of H, one per lane (lanes >= n - k hold zeros)
    uint64_t hrow[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) hrow[j] = lane < a.m ? a.rows[lane * NK + j] : 0ull;
    for (int64_t b = blockIdx.x; b < a.nblocks; b += gridDim.x) {
        const float* row = a.llr + b * (int64_t)n;
        float x[NK];
        bool ybit[NK];
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int i = j * ORBG_WAVE + lane;
            x[j] = i < n ? row[i] : 0.0f;
            ybit[j] = i < n && x[j] > 0.0f;
            const uint64_t y = ballot(ybit[j]);
            acc += __popcll(hrow[j] & y);
        }
        const uint64_t s0 = uniform_u64(ballot((acc & 1u) != 0u));
        bool found = false;
        uint32_t q = a.budget;
        int nwin = 0;
        int m_used = 1;
        int32_t j0v = 0;
        if (s0 != 0 || a.mfit != nullptr || a.j0 != nullptr) {
            // full reliability order, exact keys
            uint64_t key[NK];
#pragma unroll
            for (int j = 0; j < NK; ++j) {
                const int i = j * ORBG_WAVE + lane;
                key[j] = i < n ? (((uint64_t)(__float_as_uint(x[j]) & 0x7fffffffu) << 32) | (uint32_t)i) : ~0ull;
            }
            bitonic_sort<NK>(key);
#pragma unroll
            for (int j = 0; j < NK; ++j) {
                const int e = lane * NK + j;          // rank e + 1
                if (e < n) {
                    const uint32_t idx = (uint32_t)key[j];
                    S.pi[e + 1] = (uint16_t)idx;
                    S.h[e + 1] = a.cols[idx];
                    S.L[e + 1] = __uint_as_float((uint32_t)(key[j] >> 32));
                }
            }
            wave_lds_sync();
            const Model md = fit_model<NK>(S, n, a.mseg, a.jdiv);
            m_used = md.m;
            j0v = (int32_t)md.J[0];
            // queries to make: the budget, at most all 2^n patterns (they hold
            // a member, so the walk ends at a hit before running out)
            const uint32_t limit = (n < 32 && a.budget > (1u << n)) ? (1u << n) : a.budget;
            if (s0 == 0) {
                found = true;
                q = 1;
            } else {
                // md.m <= a.mseg = MM
                if (MM == 1 || md.m == 1) {
                    decode_walk<1>(md, a.table, S, s0, limit, found, q, nwin);
                } else if constexpr (MM >= 2) {
                    if (MM == 2 || md.m == 2) decode_walk<MM >= 2 ? 2 : 1>(md, a.table, S, s0, limit, found, q, nwin);
                    else if (MM == 3 || md.m == 3) decode_walk<MM >= 3 ? 3 : 1>(md, a.table, S, s0, limit, found, q, nwin);
                    else decode_walk<MM >= 4 ? 4 : 1>(md, a.table, S, s0, limit, found, q, nwin);
                }
            }
        } else {
            found = true;
            q = 1;
        }
        // codeword: hard decision, the winner's ranks flipped
        bool bit[NK];
#pragma unroll
        for (int j = 0; j < NK; ++j) bit[j] = ybit[j];
        if (found) {
            for (int k = 0; k < nwin; ++k) {
                const uint32_t p = uni32(S.pi[S.win[k]]);
#pragma unroll
                for (int j = 0; j < NK; ++j)
                    if ((p >> 6) == (uint32_t)j) bit[j] ^= (uint32_t)lane == (p & 63u);
            }
        }
        uint8_t* cw = a.cw + b * (int64_t)n;
#pragma unroll
        for (int j = 0; j < NK; ++j) {
            const int i = j * ORBG_WAVE + lane;
            if (i < n) cw[i] = bit[j] ? 1 : 0;
        }
        if (lane == 0) {
            a.queries[b] = found ? (uint64_t)q : (uint64_t)a.budget;
            a.abandoned[b] = found ? 0 : 1;
            if (a.mfit != nullptr) a.mfit[b] = m_used;
            if (a.j0 != nullptr) a.j0[b] = j0v;
        }
        wave_lds_sync();
    }
}

}  // namespace

template <int MM>
hipError_t launch_mline_m(const MlineArgs& a, int grid, hipStream_t stream)
{
    if (a.n <= ORBG_WAVE) mline_kernel<1, MM><<<grid, ORBG_WAVE, 0, stream>>>(a);
    else if (a.n <= 2 * ORBG_WAVE) mline_kernel<2, MM><<<grid, ORBG_WAVE, 0, stream>>>(a);
    else if (a.n <= 4 * ORBG_WAVE) mline_kernel<4, MM><<<grid, ORBG_WAVE, 0, stream>>>(a);
    else mline_kernel<8, MM><<<grid, ORBG_WAVE, 0, stream>>>(a);
    return hipGetLastError();
}

}  // namespace orbg
