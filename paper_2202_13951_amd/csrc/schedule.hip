// Query schedule of basic ORBGRAND, built on the device.
//
// The order in which putative noise patterns are tested does not depend on
// the received block: only the reliability permutation does.  Patterns are
// sets of reliability ranks 1 <= v_1 < ... < v_w <= n, taken by increasing
// logistic weight W = sum v_i (Sec. III-B, eqs. (lw), (znwl)), inside one W by
// increasing Hamming weight w (the union order of eq. (fractionation)), and
// inside one (W, w) in the order of the Landslide generator (Sec. III-C,
// Algorithm 2), which is the lexicographic order of v.  The schedule holds the
// first `len` patterns once per (n, len) and every block of every decode call
// reads it.  An entry is 8 bytes: byte 0 is a mask of the flipped ranks among
// 1..8 (bit j = rank j + 1; the decoder resolves it through a per-block table of
// the syndromes of all 256 subsets of the eight least reliable bits), bytes 1..7
// are the flipped ranks above 8 in increasing order, 0 marking an unused slot.
// A pattern of logistic weight at most 99 never flips more than seven ranks
// above 8 (9 + 10 + ... + 16 = 100); at logistic weight 100 only {9, ..., 16}
// flips eight, and it is the last pattern of its class (W = 100, w = 8: the
// lexicographically largest), so the schedule runs up to the pattern before it:
// all patterns of logistic weight <= 99 (4,827,382 for n >= 99) and those of
// weight 100 with w <= 7 and the first ones with w = 8, which covers the paper's
// abandonment threshold of 5 x 10^6 queries (Sec. IV-A) for every n >= 100.
//
// Built by three kernels:
//   1. class_count_kernel: w-subsets of {1..n} with sum W (a subset-sum count),
//      then the start offset of every non-empty class (W, w) in the order;
//   2. class_fill_kernel: one thread per class, walks the class in
//      lexicographic order by a successor rule and writes its entries;
//   3. batch_width_kernel: the largest number of ranks above 8 inside each batch
//      of 64 consecutive entries (the trip count of the decode kernel's XOR loop).
#include "orbg_device.h"
#include "orbg_internal.h"

#include <algorithm>
#include <stdint.h>
#include <vector>

namespace orbg {

// N[w][W] = number of w-subsets of {1..n} with sum W (w <= ORBG_WMAX_H,
// W <= ORBG_WCAP): the 0/1 knapsack recursion over the values v = 1..n, one
// thread per W.  Called by all ORBG_WCAP + 1 threads of the block.
__device__ void subset_counts(int n, uint64_t (*N)[ORBG_WCAP + 1])
{
    const int W = threadIdx.x;
#pragma unroll
    for (int w = 0; w <= ORBG_WMAX_H; ++w) N[w][W] = (w == 0 && W == 0) ? 1ull : 0ull;
    __syncthreads();
    const int vmax = n < ORBG_WCAP ? n : ORBG_WCAP;
    for (int v = 1; v <= vmax; ++v) {
        const int wtop = v < ORBG_WMAX_H ? v : ORBG_WMAX_H;
        for (int w = wtop; w >= 1; --w) {
            const uint64_t add = (W >= v) ? N[w - 1][W - v] : 0ull;
            N[w][W] += add;
            __syncthreads();
        }
    }
}

// counts layout: [ORBG_WMAX_H + 1][ORBG_WCAP + 1]
__global__ void __launch_bounds__(ORBG_WCAP + 1)
class_count_kernel(int n, uint64_t len, ClassInfo* classes, int* nclass_out, int* wlast_out)
{
    __shared__ uint64_t N[ORBG_WMAX_H + 1][ORBG_WCAP + 1];
    subset_counts(n, N);
    const int W = threadIdx.x;
    if (W != 0) return;
    // lay the classes out: W ascending, w ascending, until len entries exist
    uint64_t off = 0;
    int nc = 0, wlast = 0;
    for (int Wl = 0; Wl <= ORBG_WLEVEL_SCHED && off < len; ++Wl) {
        for (int w = 0; w <= ORBG_WMAX_H && off < len; ++w) {
            uint64_t c = N[w][Wl];
            if (Wl > ORBG_WLEVEL_PACKED) {
                // weight 100: classes up to w = 8 without its last pattern {9..16}
                // (present when n >= 16); what follows it cannot be represented
                if (w > ORBG_HIGH_SLOTS + 1) break;
                if (w == ORBG_HIGH_SLOTS + 1 && n >= 16) c -= 1;
            }
            if (c == 0) continue;
            classes[nc].W = Wl;
            classes[nc].w = w;
            classes[nc].offset = off;
            classes[nc].count = c;
            ++nc;
            off += c;
            wlast = Wl;
        }
    }
    // off < len here means the schedule would need a pattern it cannot hold
    *nclass_out = (off >= len) ? nc : -nc - 1;
    *wlast_out = wlast;
}

// Largest sum of `cnt` distinct values in [1, n]: n + (n-1) + ... (cnt terms).
__device__ __forceinline__ int max_sum(int cnt, int n) { return cnt * n - cnt * (cnt - 1) / 2; }
// Smallest sum of `cnt` distinct values all greater than x.
__device__ __forceinline__ int min_sum_above(int cnt, int x) { return cnt * x + cnt * (cnt + 1) / 2; }

// Lexicographically smallest strictly increasing fill of v[p..w-1], values in
// [lo, n], summing to rem.  Caller guarantees feasibility.
__device__ __forceinline__ void smallest_fill(int* v, int p, int w, int lo, int rem, int n)
{
    for (int i = p; i < w; ++i) {
        const int after = w - 1 - i;                 // elements still to place after v[i]
        int x = rem - max_sum(after, n);             // the rest can absorb at most max_sum
        if (x < lo) x = lo;
        v[i] = x;
        rem -= x;
        lo = x + 1;
    }
}

__device__ __forceinline__ void store_entry(uint2* out, const int* v, int w)
{
    uint64_t e = 0;
    int slot = 1;
    for (int i = 0; i < w; ++i) {
        if (v[i] <= ORBG_LOW_RANKS) e |= 1ull << (v[i] - 1);
        else e |= (uint64_t)v[i] << (8 * slot++);
    }
    *out = make_uint2((uint32_t)e, (uint32_t)(e >> 32));
}

__global__ void class_fill_kernel(int n, uint64_t len, const ClassInfo* classes, int nclass,
                                  uint2* entries)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nclass) return;
    const int W = classes[c].W, w = classes[c].w;
    uint64_t g = classes[c].offset;
    const uint64_t end = classes[c].offset + classes[c].count;
    int v[ORBG_WMAX_H];
    if (w == 0) {                                     // the empty pattern
        if (g < len) entries[g] = make_uint2(0u, 0u);
        return;
    }
    smallest_fill(v, 0, w, 1, W, n);
    for (; g < end && g < len; ++g) {
        store_entry(entries + g, v, w);
        // successor: the right-most position p < w-1 that can grow by one while
        // the positions after it still admit a strictly increasing fill
        int prefix = 0;
        for (int i = 0; i < w; ++i) prefix += v[i];
        int p = w - 2;
        for (; p >= 0; --p) {
            prefix -= v[p + 1];                       // prefix = sum v[0..p]
            const int x = v[p] + 1;
            const int rem = W - (prefix - v[p]) - x;  // what positions p+1.. must hold
            const int after = w - 1 - p;
            if (x <= n && rem >= min_sum_above(after, x) && rem <= max_sum(after, n)) {
                v[p] = x;
                smallest_fill(v, p + 1, w, x + 1, rem, n);
                break;
            }
        }
        if (p < 0) break;
    }
}

// Deepest rank referenced by the first `len` entries (one thread per batch of
// 64), and by the first batch alone (rmax[1]).
__global__ void rank_depth_kernel(const uint2* entries, uint64_t len, uint64_t nbatch, int* rmax)
{
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbatch) return;
    int r = 0;
    for (uint64_t g = b * 64; g < b * 64 + 64 && g < len; ++g) {
        const uint2 e2 = entries[g];
        const uint64_t e = ((uint64_t)e2.y << 32) | e2.x;
        for (int i = 1; i <= ORBG_HIGH_SLOTS; ++i) {
            const int rk = (int)((e >> (8 * i)) & 0xff);
            r = rk > r ? rk : r;
        }
        const int low = (int)(e & 0xff);
        if (low) {
            const int top = 32 - __clz(low);          // highest set bit + 1 = rank
            r = top > r ? top : r;
        }
    }
    atomicMax(rmax, r);
    if (b == 0) rmax[1] = r;
}

__global__ void unpack_kernel(const uint2* entries, uint64_t count, uint8_t* out)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= count) return;
    const uint2 e2 = entries[g];
    const uint64_t e = ((uint64_t)e2.y << 32) | e2.x;
    uint8_t row[16] = {0};
    int w = 0;
    for (int j = 0; j < ORBG_LOW_RANKS; ++j)
        if ((e >> j) & 1) row[w++] = (uint8_t)(j + 1);
    for (int i = 1; i <= ORBG_HIGH_SLOTS; ++i) {
        const int rk = (int)((e >> (8 * i)) & 0xff);
        if (rk) row[w++] = (uint8_t)rk;
    }
    for (int i = 0; i < 16; ++i) out[g * 16 + i] = row[i];
}

// Builds the schedule of the first `len` patterns for length n on `stream`.
// Blocks until the class layout is known (one small device-to-host copy).
int orbg_build_schedule(int n, uint64_t len, hipStream_t stream, Schedule* out, char* err, size_t errlen)
{
    ClassInfo* d_classes = nullptr;
    int* d_small = nullptr;
    const int max_classes = (ORBG_WCAP + 1) * (ORBG_WMAX_H + 1);
    if (hipMalloc(&d_classes, sizeof(ClassInfo) * max_classes) != hipSuccess ||
        hipMalloc(&d_small, sizeof(int) * 4) != hipSuccess) {
        snprintf(err, errlen, "schedule: device allocation failed");
        (void)hipFree(d_classes); (void)hipFree(d_small);
        return -2;
    }
    (void)hipMemsetAsync(d_small, 0, sizeof(int) * 4, stream);
    class_count_kernel<<<1, ORBG_WCAP + 1, 0, stream>>>(n, len, d_classes, d_small, d_small + 1);
    int host_small[2] = {0, 0};
    (void)hipMemcpyAsync(host_small, d_small, sizeof(int) * 2, hipMemcpyDeviceToHost, stream);
    if (hipStreamSynchronize(stream) != hipSuccess) {
        snprintf(err, errlen, "schedule: class count kernel failed: %s", hipGetErrorString(hipGetLastError()));
        (void)hipFree(d_classes); (void)hipFree(d_small);
        return -3;
    }
    int nclass = host_small[0];
    if (nclass < 0) {
        snprintf(err, errlen, "schedule: %llu patterns reach past the pattern {9, ..., 16} of logistic "
                 "weight %d", (unsigned long long)len, ORBG_WLEVEL_SCHED);
        (void)hipFree(d_classes); (void)hipFree(d_small);
        return -1;
    }
    const uint64_t nbatch = (len + 63) / 64;
    uint2* d_entries = nullptr;
    // ORBG_SCHED_PAD zero batches follow the last one, so a search may load the
    // entries of a few steps past its end without a bounds check
    const uint64_t alloc = (nbatch + ORBG_SCHED_PAD) * 64;
    if (hipMalloc(&d_entries, sizeof(uint2) * alloc) != hipSuccess) {
        snprintf(err, errlen, "schedule: cannot allocate %llu entries", (unsigned long long)len);
        (void)hipFree(d_classes); (void)hipFree(d_small);
        return -2;
    }
    // entries past len (up to the batch boundary) stay zero: the empty pattern
    (void)hipMemsetAsync(d_entries, 0, sizeof(uint2) * alloc, stream);
    class_fill_kernel<<<(nclass + 63) / 64, 64, 0, stream>>>(n, len, d_classes, nclass, d_entries);
    rank_depth_kernel<<<(unsigned)((nbatch + 255) / 256), 256, 0, stream>>>(d_entries, len, nbatch, d_small + 2);
    int rmax[2] = {0, 0};
    (void)hipMemcpyAsync(rmax, d_small + 2, sizeof(int) * 2, hipMemcpyDeviceToHost, stream);
    if (hipStreamSynchronize(stream) != hipSuccess) {
        snprintf(err, errlen, "schedule: fill kernels failed: %s", hipGetErrorString(hipGetLastError()));
        (void)hipFree(d_entries); (void)hipFree(d_classes); (void)hipFree(d_small);
        return -3;
    }
    (void)hipFree(d_classes);
    (void)hipFree(d_small);
    out->n = n;
    out->len = len;
    out->entries = d_entries;
    out->nbatch = nbatch;
    out->rmax = rmax[0];
    out->rmax0 = rmax[1];
    out->wlast = host_small[1];
    return 0;
}

int orbg_unpack_schedule(const Schedule* s, uint64_t count, uint8_t* d_out, hipStream_t stream)
{
    if (count > s->len) return -1;
    unpack_kernel<<<(unsigned)((count + 255) / 256), 256, 0, stream>>>(s->entries, count, d_out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---------------------------------------------------------------------------
// 1-line ORBGRAND schedules.  With one segment of slope beta = 1 and offset J0
// (Sec. III-D eq. (relest_seg) and Sec. III-E eq. (quant) with m = 1), the reliability weight
// of a pattern of Hamming weight w and logistic weight W is J0 w + W
// (eq. (W2IJ)), so the 1-line order takes the same (W, w) classes as the basic
// order, each still in Landslide (lexicographic) order, but sorted by
// (J0 w + W, w).  One schedule per J0 in [-1, j0max] is built, J0 = -1 first,
// each `stride` entries apart.
//
// j0max: for J0 at least the largest W among the first len patterns of the
// order that takes Hamming weight first (then W, then lexicographic order),
// every J0 gives that same prefix (a pattern p of that prefix and any pattern q
// of larger Hamming weight satisfy J0 (w_q - w_p) + W_q - W_p > 0), so larger
// fitted values decode with the schedule of j0max.

__global__ void __launch_bounds__(ORBG_WCAP + 1) subset_count_kernel(int n, uint64_t* out)
{
    __shared__ uint64_t N[ORBG_WMAX_H + 1][ORBG_WCAP + 1];
    subset_counts(n, N);
    for (int w = 0; w <= ORBG_WMAX_H; ++w) out[w * (ORBG_WCAP + 1) + threadIdx.x] = N[w][threadIdx.x];
}

static int64_t host_max_sum(int w, int n) { return (int64_t)w * n - (int64_t)w * (w - 1) / 2; }

// Class layout of every J0 schedule from the subset counts N (host side).
static int layout_1line(int n, uint64_t len, uint64_t stride, const uint64_t* N, std::vector<ClassInfo>& out,
                        int* j0max, char* err, size_t errlen)
{
    auto cnt = [&](int w, int W) { return N[w * (ORBG_WCAP + 1) + W]; };
    const int wtop = n < ORBG_WMAX_H ? n : ORBG_WMAX_H;
    // largest W of the first len patterns in Hamming-weight-first order
    uint64_t off = 0;
    int wmaxW = 0;
    for (int w = 0; w <= wtop && off < len; ++w) {
        for (int W = 0; W <= ORBG_WCAP && off < len; ++W)
            if (cnt(w, W)) { off += cnt(w, W); wmaxW = W > wmaxW ? W : wmaxW; }
        if (off < len && host_max_sum(w, n) > ORBG_WCAP) {
            snprintf(err, errlen, "1-line schedule: %llu patterns of Hamming weight <= %d need logistic weights "
                     "above %d", (unsigned long long)len, w, ORBG_WCAP);
            return -1;
        }
    }
    if (off < len) {
        snprintf(err, errlen, "1-line schedule: %llu patterns need Hamming weights above %d",
                 (unsigned long long)len, ORBG_WMAX_H);
        return -1;
    }
    *j0max = wmaxW;
    struct Cls { int64_t cost; int w; int W; };
    std::vector<Cls> cls;
    for (int J = -1; J <= wmaxW; ++J) {
        cls.clear();
        for (int w = 0; w <= wtop; ++w)
            for (int W = 0; W <= ORBG_WCAP; ++W)
                if (cnt(w, W)) cls.push_back({(int64_t)J * w + W, w, W});
        std::sort(cls.begin(), cls.end(), [](const Cls& a, const Cls& b) {
            return a.cost != b.cost ? a.cost < b.cost : a.w < b.w;
        });
        // the cheapest class the counts do not hold (W > WCAP or w > WMAX_H)
        int64_t missing = INT64_MAX;
        for (int w = 1; w <= n; ++w) {
            const int64_t lo = (int64_t)w * (w + 1) / 2;
            int64_t W0 = -1;
            if (w > ORBG_WMAX_H) W0 = lo;
            else if (host_max_sum(w, n) > ORBG_WCAP) W0 = lo > ORBG_WCAP + 1 ? lo : ORBG_WCAP + 1;
            if (W0 >= 0 && (int64_t)J * w + W0 < missing) missing = (int64_t)J * w + W0;
        }
        const uint64_t base = (uint64_t)(J + 1) * stride;
        uint64_t o = 0;
        int64_t last = 0;
        for (const Cls& c : cls) {
            if (o >= len) break;
            if (c.w > ORBG_HIGH_SLOTS && c.W > ORBG_WLEVEL_PACKED) {
                snprintf(err, errlen, "1-line schedule (J0 = %d): class W = %d, w = %d does not fit an entry", J, c.W,
                         c.w);
                return -1;
            }
            const uint64_t take = cnt(c.w, c.W) < len - o ? cnt(c.w, c.W) : len - o;
            out.push_back({c.W, c.w, base + o, take});
            o += take;
            last = c.cost;
        }
        if (o < len || last >= missing) {
            snprintf(err, errlen, "1-line schedule (J0 = %d): %llu patterns reach logistic weights above %d", J,
                     (unsigned long long)len, ORBG_WCAP);
            return -1;
        }
    }
    return 0;
}

int orbg_build_schedule_1line(int n, uint64_t len, hipStream_t stream, Schedule1* out, char* err, size_t errlen)
{
    const int WN = (ORBG_WMAX_H + 1) * (ORBG_WCAP + 1);
    uint64_t* d_counts = nullptr;
    int* d_small = nullptr;
    if (hipMalloc(&d_counts, sizeof(uint64_t) * WN) != hipSuccess || hipMalloc(&d_small, sizeof(int) * 4) != hipSuccess) {
        snprintf(err, errlen, "1-line schedule: device allocation failed");
        (void)hipFree(d_counts); (void)hipFree(d_small);
        return -2;
    }
    std::vector<uint64_t> N(WN);
    subset_count_kernel<<<1, ORBG_WCAP + 1, 0, stream>>>(n, d_counts);
    (void)hipMemcpyAsync(N.data(), d_counts, sizeof(uint64_t) * WN, hipMemcpyDeviceToHost, stream);
    if (hipStreamSynchronize(stream) != hipSuccess) {
        snprintf(err, errlen, "1-line schedule: count kernel failed: %s", hipGetErrorString(hipGetLastError()));
        (void)hipFree(d_counts); (void)hipFree(d_small);
        return -3;
    }
    (void)hipFree(d_counts);
    const uint64_t nbatch = (len + 63) / 64;
    const uint64_t stride = (nbatch + ORBG_SCHED_PAD) * 64;
    std::vector<ClassInfo> classes;
    int j0max = 0;
    int rc = layout_1line(n, len, stride, N.data(), classes, &j0max, err, errlen);
    if (rc != 0) { (void)hipFree(d_small); return rc; }
    const uint64_t total = (uint64_t)(j0max + 2) * stride;
    ClassInfo* d_classes = nullptr;
    uint2* d_entries = nullptr;
    if (hipMalloc(&d_classes, sizeof(ClassInfo) * classes.size()) != hipSuccess ||
        hipMalloc(&d_entries, sizeof(uint2) * total) != hipSuccess) {
        snprintf(err, errlen, "1-line schedule: cannot allocate %d schedules of %llu entries", j0max + 2,
                 (unsigned long long)stride);
        (void)hipFree(d_classes); (void)hipFree(d_entries); (void)hipFree(d_small);
        return -2;
    }
    (void)hipMemcpyAsync(d_classes, classes.data(), sizeof(ClassInfo) * classes.size(), hipMemcpyHostToDevice, stream);
    (void)hipMemsetAsync(d_small, 0, sizeof(int) * 4, stream);
    (void)hipMemsetAsync(d_entries, 0, sizeof(uint2) * total, stream);
    const int nclass = (int)classes.size();
    class_fill_kernel<<<(nclass + 63) / 64, 64, 0, stream>>>(n, total, d_classes, nclass, d_entries);
    rank_depth_kernel<<<(unsigned)((total / 64 + 255) / 256), 256, 0, stream>>>(d_entries, total, total / 64,
                                                                                 d_small);
    int rmax[2] = {0, 0};
    (void)hipMemcpyAsync(rmax, d_small, sizeof(int) * 2, hipMemcpyDeviceToHost, stream);
    if (hipStreamSynchronize(stream) != hipSuccess) {
        snprintf(err, errlen, "1-line schedule: fill kernels failed: %s", hipGetErrorString(hipGetLastError()));
        (void)hipFree(d_classes); (void)hipFree(d_entries); (void)hipFree(d_small);
        return -3;
    }
    (void)hipFree(d_classes);
    (void)hipFree(d_small);
    out->n = n;
    out->len = len;
    out->nbatch = nbatch;
    out->stride = stride;
    out->j0max = j0max;
    out->entries = d_entries;
    out->rmax = rmax[0];
    return 0;
}

int orbg_unpack_entries(const uint2* entries, uint64_t count, uint8_t* d_out, hipStream_t stream)
{
    unpack_kernel<<<(unsigned)((count + 255) / 256), 256, 0, stream>>>(entries, count, d_out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace orbg
