// Learned batch-order proposal: a 128 -> 256 -> 256 -> 64 ReLU network in BF16
// with FP32 accumulation on the matrix cores, its backward pass and Adam.
//
// Input of the network: a block's reliabilities |LLR_i| sorted ascending (the
// ordered reliability curve of Sec. III-A), scaled by 1/8 and rounded to BF16.
// Output: 64 logits, one per batch of 64 consecutive patterns of the basic
// ORBGRAND order; the decoder tests batches by decreasing logit
// (orbg_decode_ordered) and falls back to the plain order after them.
//
// Parameters (FP32 masters, flat): W1 [256 x 128], b1 [256], W2 [256 x 256],
// b2 [256], W3 [64 x 256], b3 [64] (output x input, row-major).  The forward
// uses BF16 copies of the weights (same layout); the backward also uses BF16
// transposed copies W1t [128 x 256], W2t [256 x 256], W3t [256 x 64].
//
// GEMMs: gfx950's v_mfma_f32_16x16x32_bf16 tiles, a 64 x 64 output tile per
// 256-thread workgroup (each wave 32 x 32 = 2 x 2 MFMA tiles), K in steps of 32
// with 8-value fragments read straight from global memory (operands are small
// and stay in L2).  Weight gradients reduce over the batch: split-K partials in
// FP32 and a deterministic reduction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "orbg_device.h"
#include "orbg_mlp.h"

namespace orbg {

typedef short s8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);                 // nearest, ties to even
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// Features: sorted |LLR| / 8 in BF16, one wave per block (n = 128).  ids (or
// nullptr): row ids[b] of llr gives feature row b.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) features_kernel(const float* __restrict__ llr, int64_t batch,
                                                       uint16_t* __restrict__ x, const int64_t* __restrict__ ids)
{
    const int lane = lane_id();
    const int64_t b = (int64_t)blockIdx.x * 4 + threadIdx.x / ORBG_WAVE;
    if (b >= batch) return;
    const int64_t src = ids ? ids[b] : b;
    uint32_t key[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) key[j] = __float_as_uint(llr[src * MLP_IN + j * ORBG_WAVE + lane]) & 0x7fffffffu;
    bitonic_sort<2, uint32_t>(key);
#pragma unroll
    for (int j = 0; j < 2; ++j) x[b * MLP_IN + lane * 2 + j] = f32_to_bf16(__uint_as_float(key[j]) * 0.125f);
}

// ---------------------------------------------------------------------------
// GEMM C[M x N] = sum_k A(i, k) B(k, j); A(i, k) = A[i * a_i + k * a_k],
// B(k, j) = B[k * b_k + j * b_j] (BF16).  AK / BK: unit stride along k.
// ---------------------------------------------------------------------------
enum { EPI_HIDDEN = 0, EPI_LOGITS = 1, EPI_MASKED = 2, EPI_PARTIAL = 3 };

// Eight consecutive-k values of one row (A) or column (B); `nk` of them exist
// (0..8).  UNIT: unit stride, then the caller guarantees nk is 0 or 8.
template <bool UNIT>
__device__ __forceinline__ s8v load_frag(const uint16_t* __restrict__ p, int64_t stride, int nk)
{
    s8v r = {0, 0, 0, 0, 0, 0, 0, 0};
    if (nk <= 0) return r;
    if (UNIT) {
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        r[0] = (short)(v.x & 0xffffu); r[1] = (short)(v.x >> 16);
        r[2] = (short)(v.y & 0xffffu); r[3] = (short)(v.y >> 16);
        r[4] = (short)(v.z & 0xffffu); r[5] = (short)(v.z >> 16);
        r[6] = (short)(v.w & 0xffffu); r[7] = (short)(v.w >> 16);
    } else {
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (t < nk) r[t] = (short)p[t * stride];
    }
    return r;
}

template <bool AK, bool BK, int EPI>
__global__ void __launch_bounds__(256)
gemm_kernel(const uint16_t* __restrict__ A, int64_t a_i, int64_t a_k, const uint16_t* __restrict__ B, int64_t b_k,
            int64_t b_j, int M, int N, int K, int kchunk, const float* __restrict__ bias,
            void* __restrict__ out, int64_t ldo, const uint16_t* __restrict__ mask, int64_t ldm)
{
    const int lane = lane_id();
    const int wave = threadIdx.x / ORBG_WAVE;
    const int i0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int j0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int r = lane & 15, q = lane >> 4;
    f4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = (f4v){0.f, 0.f, 0.f, 0.f};
    for (int k = kb; k < ke; k += 32) {
        const int kk = k + 8 * q;                   // this lane's 8 consecutive k
        const int nk = min(8, ke - kk);             // how many of them exist (<= 0: none)
        s8v fa[2], fb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int i = i0 + a * 16 + r;
            fa[a] = load_frag<AK>(A + (int64_t)i * a_i + (int64_t)kk * a_k, a_k, i < M ? nk : 0);
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int j = j0 + c * 16 + r;
            fb[c] = load_frag<BK>(B + (int64_t)j * b_j + (int64_t)kk * b_k, b_k, j < N ? nk : 0);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, fa[a]),
                                                                    __builtin_bit_cast(bf8v, fb[c]), acc[a][c], 0, 0, 0);
    }
    // lane holds D[4q + t][r] of each 16 x 16 tile, t = 0..3
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = i0 + a * 16 + 4 * q + t;
                const int j = j0 + c * 16 + r;
                if (i >= M || j >= N) continue;
                const float v = acc[a][c][t];
                if (EPI == EPI_HIDDEN) {
                    reinterpret_cast<uint16_t*>(out)[(int64_t)i * ldo + j] = f32_to_bf16(fmaxf(v + bias[j], 0.f));
                } else if (EPI == EPI_LOGITS) {
                    reinterpret_cast<float*>(out)[(int64_t)i * ldo + j] = v + bias[j];
                } else if (EPI == EPI_MASKED) {
                    const bool on = mask[(int64_t)i * ldm + j] != 0;      // ReLU output > 0
                    reinterpret_cast<uint16_t*>(out)[(int64_t)i * ldo + j] = on ? f32_to_bf16(v) : (uint16_t)0;
                } else {
                    reinterpret_cast<float*>(out)[(int64_t)blockIdx.z * M * N + (int64_t)i * N + j] = v;
                }
            }
}

// out[e] = sum over s < splits of part[s * count + e]
__global__ void reduce_partials_kernel(const float* __restrict__ part, int splits, int64_t count,
                                       float* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * count + e];
    out[e] = s;
}

// Column sums of a BF16 [rows x cols] matrix: part[z * cols + j] over rows [z*chunk, ...).
__global__ void colsum_kernel(const uint16_t* __restrict__ g, int64_t rows, int cols, int64_t chunk,
                              float* __restrict__ part)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    if (j >= cols) return;
    const int64_t rb = (int64_t)z * chunk, re = min(rows, rb + chunk);
    float s = 0.f;
    for (int64_t i = rb; i < re; ++i) s += bf16_to_f32(g[i * cols + j]);
    part[(int64_t)z * cols + j] = s;
}

// Softmax cross-entropy, one wave per row (lane = class): dl = (softmax - onehot) / B
// in BF16, per-row loss into rowloss.
__global__ void __launch_bounds__(256) softmax_ce_kernel(const float* __restrict__ logits,
                                                         const int32_t* __restrict__ labels, int64_t batch,
                                                         uint16_t* __restrict__ dl, float* __restrict__ rowloss)
{
    const int lane = lane_id();
    const int64_t b = (int64_t)blockIdx.x * 4 + threadIdx.x / ORBG_WAVE;
    if (b >= batch) return;
    const float v = logits[b * MLP_OUT + lane];
    float mx = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) mx = fmaxf(mx, __shfl_xor(mx, d, ORBG_WAVE));
    const float e = __expf(v - mx);
    float s = e;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) s += __shfl_xor(s, d, ORBG_WAVE);
    const int lab = labels[b];
    const float p = e / s;
    dl[b * MLP_OUT + lane] = f32_to_bf16((p - (lane == lab ? 1.f : 0.f)) / (float)batch);
    const float vl = __shfl(v, lab & 63, ORBG_WAVE);
    if (lane == 0) rowloss[b] = (__logf(s) + mx - vl);
}

__global__ void sum_kernel(const float* __restrict__ x, int64_t count, float scale, float* __restrict__ out)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < count; i += 256) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// BF16 copies (and transposed copies of the weight matrices) of FP32 masters.
__device__ __forceinline__ void write_copies(int64_t p, float w, uint16_t* __restrict__ wb, uint16_t* __restrict__ wt)
{
    const uint16_t h = f32_to_bf16(w);
    wb[p] = h;
    if (p < MLP_OFF_B1) {                                           // W1 [256 x 128]
        const int64_t rr = p / MLP_IN, cc = p % MLP_IN;
        wt[MLP_T_W1 + cc * MLP_HID + rr] = h;
    } else if (p >= MLP_OFF_W2 && p < MLP_OFF_B2) {                 // W2 [256 x 256]
        const int64_t qq = p - MLP_OFF_W2, rr = qq / MLP_HID, cc = qq % MLP_HID;
        wt[MLP_T_W2 + cc * MLP_HID + rr] = h;
    } else if (p >= MLP_OFF_W3 && p < MLP_OFF_B3) {                 // W3 [64 x 256]
        const int64_t qq = p - MLP_OFF_W3, rr = qq / MLP_HID, cc = qq % MLP_HID;
        wt[MLP_T_W3 + cc * MLP_OUT + rr] = h;
    }
}

__global__ void prepare_kernel(const float* __restrict__ w, uint16_t* __restrict__ wb, uint16_t* __restrict__ wt)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_NPARAM) write_copies(p, w[p], wb, wt);
}

__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, float lr, float beta1, float beta2, float eps, float c1,
                            float c2, uint16_t* __restrict__ wb, uint16_t* __restrict__ wt)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float gg = g[p];
    const float mm = beta1 * m[p] + (1.f - beta1) * gg;
    const float vv = beta2 * v[p] + (1.f - beta2) * gg * gg;
    m[p] = mm;
    v[p] = vv;
    const float ww = w[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    w[p] = ww;
    write_copies(p, ww, wb, wt);
}

// One row's batch order (one logit per lane, all lanes active): lane e
// returns the e-th batch to test.
__device__ __forceinline__ uint8_t order_of_row(float logit, int pin0)
{
    const int lane = lane_id();
    const float f = logit + 0.0f;                               // -0 -> +0
    const uint32_t u = __float_as_uint(f);
    const bool nan = (u & 0x7fffffffu) > 0x7f800000u;
    const uint32_t up = nan ? 0u : ((u >> 31) ? ~u : (u | 0x80000000u));   // increasing with f, NaN lowest
    uint64_t key[1] = {((uint64_t)(~up) << 32) | (uint32_t)lane};          // ascending = decreasing f
    if (pin0 && lane == 0) key[0] = 0ull;
    bitonic_sort<1, uint64_t>(key);
    return (uint8_t)(key[0] & 63u);
}

// Batch order: decreasing logit, ties (and +-0) to the lower index, NaN last;
// pin0: batch 0 first whatever its logit, the others as before.  One wave per
// row: key = (order-preserving bits of -logit) << 32 | index, sorted ascending
// by the register bitonic network; lane e then holds the e-th batch to test.
__global__ void __launch_bounds__(256) order_kernel(const float* __restrict__ logits, int64_t batch,
                                                    uint8_t* __restrict__ order, int pin0)
{
    const int lane = lane_id();
    const int64_t b = (int64_t)blockIdx.x * 4 + threadIdx.x / ORBG_WAVE;
    if (b >= batch) return;
    order[b * MLP_OUT + lane] = order_of_row(logits[b * MLP_OUT + lane], pin0);
}

// Order table of a gated decode: row b = identity for blocks decided by batch 0,
// the learned order for listed blocks (row ids[i] = rows[i]).
__global__ void order_identity_kernel(uint8_t* __restrict__ order, int64_t batch)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < batch * MLP_OUT) order[e] = (uint8_t)(e % MLP_OUT);
}

__global__ void order_scatter_kernel(const uint8_t* __restrict__ rows, const int64_t* __restrict__ ids, int64_t count,
                                     uint8_t* __restrict__ order)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count * MLP_OUT) order[ids[e / MLP_OUT] * MLP_OUT + e % MLP_OUT] = rows[e];
}

hipError_t mlp_order_table(const uint8_t* rows, const int64_t* ids, int64_t count, int64_t batch, uint8_t* order,
                           hipStream_t st)
{
    if (batch > 0)
        order_identity_kernel<<<(unsigned)((batch * MLP_OUT + 255) / 256), 256, 0, st>>>(order, batch);
    if (count > 0)
        order_scatter_kernel<<<(unsigned)((count * MLP_OUT + 255) / 256), 256, 0, st>>>(rows, ids, count, order);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused inference: (features,) the three layers and (the batch order) of
// FT = 32 rows per 256-thread workgroup.  The rows' features and hidden
// activations stay in LDS as BF16 [row][k], the 16-byte groups of a row
// XOR-swizzled by the row index so that the 16 rows an MFMA fragment reads
// fall in different banks; each wave computes a quarter of a layer's outputs
// for all FT rows, its weight fragments read straight from global memory (the
// BF16 weights, 224 KB, stay in L2).  Per output the k loop, the MFMA shape
// and the epilogue are those of gemm_kernel, so the logits equal the unfused
// forward's bit for bit.
// ---------------------------------------------------------------------------
constexpr int FT = 32;

// Element offset of (row, k) in a swizzled [FT][kdim] activation tile.
__device__ __forceinline__ int swz(int row, int k, int kdim)
{
    return row * kdim + ((((k >> 3) ^ (row & 15))) << 3) + (k & 7);
}

// One layer: out(i, j) = sum_k in(i, k) W[j][k] for the FT rows and this
// wave's N / 4 outputs.  HIDDEN: BF16(ReLU(. + bias)) to the swizzled LDS tile
// `oh`; else . + bias as FP32 to `of` (row stride MLP_OUT).
template <int K, int N, bool HIDDEN>
__device__ __forceinline__ void fused_layer(const uint16_t* in, const uint16_t* __restrict__ W,
                                            const float* __restrict__ bias, uint16_t* oh, float* of)
{
    const int lane = lane_id();
    const int wave = threadIdx.x / ORBG_WAVE;
    const int r = lane & 15, q = lane >> 4;
    constexpr int NW = N / 4, CT = NW / 16, RT = FT / 16;
    f4v acc[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[a][c] = (f4v){0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k = 0; k < K; k += 32) {
        const int kk = k + 8 * q;
        s8v fa[RT], fb[CT];
#pragma unroll
        for (int a = 0; a < RT; ++a) fa[a] = *reinterpret_cast<const s8v*>(in + swz(a * 16 + r, kk, K));
#pragma unroll
        for (int c = 0; c < CT; ++c)
            fb[c] = *reinterpret_cast<const s8v*>(W + (int64_t)(wave * NW + c * 16 + r) * K + kk);
#pragma unroll
        for (int a = 0; a < RT; ++a)
#pragma unroll
            for (int c = 0; c < CT; ++c)
                acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, fa[a]),
                                                                    __builtin_bit_cast(bf8v, fb[c]), acc[a][c], 0, 0, 0);
    }
    // lane holds D[4q + t][r] of each 16 x 16 tile, t = 0..3
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = a * 16 + 4 * q + t;
                const int j = wave * NW + c * 16 + r;
                const float v = acc[a][c][t];
                if (HIDDEN) oh[swz(i, j, N)] = f32_to_bf16(fmaxf(v + bias[j], 0.f));
                else of[i * MLP_OUT + j] = v + bias[j];
            }
}

// FEAT: features of llr rows (ids[b], or b) made here, a row outside
// [0, llr_rows) giving zero features; else read from x.  logits (or nullptr)
// and order (or nullptr, ORDER false) receive the results.
template <bool FEAT, bool ORDER>
__global__ void __launch_bounds__(256)
mlp_infer_kernel(const float* __restrict__ llr, int64_t llr_rows, const int64_t* __restrict__ ids,
                 const uint16_t* __restrict__ x, int64_t batch, const float* __restrict__ w,
                 const uint16_t* __restrict__ wb, float* __restrict__ logits, uint8_t* __restrict__ order, int pin0)
{
    __shared__ __align__(16) uint16_t sa[FT * MLP_HID];     // features (FT x 128), then h2
    __shared__ __align__(16) uint16_t sb[FT * MLP_HID];     // h1, then the logits (FT x 64 FP32)
    const int lane = lane_id();
    const int wave = threadIdx.x / ORBG_WAVE;
    const int64_t row0 = (int64_t)blockIdx.x * FT;
    const int rows = (int)(batch - row0 < FT ? batch - row0 : FT);
    if (FEAT) {
        // sorted |LLR| / 8 in BF16 (as features_kernel); rows past the batch are zero
        for (int rr = wave; rr < FT; rr += 4) {
            uint32_t key[2] = {0u, 0u};
            const int64_t src = rr < rows ? (ids ? ids[row0 + rr] : row0 + rr) : -1;
            if (src >= 0 && src < llr_rows) {
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    key[j] = __float_as_uint(llr[src * MLP_IN + j * ORBG_WAVE + lane]) & 0x7fffffffu;
            }
            bitonic_sort<2, uint32_t>(key);
            const uint32_t pair = (uint32_t)f32_to_bf16(__uint_as_float(key[0]) * 0.125f) |
                                  ((uint32_t)f32_to_bf16(__uint_as_float(key[1]) * 0.125f) << 16);
            *reinterpret_cast<uint32_t*>(sa + swz(rr, 2 * lane, MLP_IN)) = pair;
        }
    } else {
        for (int g = threadIdx.x; g < FT * (MLP_IN / 8); g += 256) {
            const int rr = g / (MLP_IN / 8), kg = g % (MLP_IN / 8);
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (rr < rows) v = *reinterpret_cast<const uint4*>(x + (row0 + rr) * MLP_IN + kg * 8);
            *reinterpret_cast<uint4*>(sa + swz(rr, kg * 8, MLP_IN)) = v;
        }
    }
    __syncthreads();
    fused_layer<MLP_IN, MLP_HID, true>(sa, wb + MLP_OFF_W1, w + MLP_OFF_B1, sb, nullptr);
    __syncthreads();
    fused_layer<MLP_HID, MLP_HID, true>(sb, wb + MLP_OFF_W2, w + MLP_OFF_B2, sa, nullptr);
    __syncthreads();
    float* lg = reinterpret_cast<float*>(sb);
    fused_layer<MLP_HID, MLP_OUT, false>(sa, wb + MLP_OFF_W3, w + MLP_OFF_B3, nullptr, lg);
    __syncthreads();
    if (logits != nullptr)
        for (int e = threadIdx.x; e < rows * MLP_OUT; e += 256) logits[row0 * MLP_OUT + e] = lg[e];
    if (ORDER)
        for (int rr = wave; rr < FT; rr += 4) {
            const uint8_t o = order_of_row(lg[rr * MLP_OUT + lane], pin0);
            if (rr < rows) order[(row0 + rr) * MLP_OUT + lane] = o;
        }
}

hipError_t mlp_infer(const float* w, const uint16_t* wb, const float* llr, int64_t llr_rows, const int64_t* ids,
                     const uint16_t* x, int64_t batch, float* logits, uint8_t* order, bool pin0, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((batch + FT - 1) / FT);
    if (llr) {
        if (order)
            mlp_infer_kernel<true, true><<<grid, 256, 0, st>>>(llr, llr_rows, ids, x, batch, w, wb, logits, order, pin0);
        else
            mlp_infer_kernel<true, false><<<grid, 256, 0, st>>>(llr, llr_rows, ids, x, batch, w, wb, logits, order, pin0);
    } else {
        if (order)
            mlp_infer_kernel<false, true><<<grid, 256, 0, st>>>(llr, llr_rows, ids, x, batch, w, wb, logits, order, pin0);
        else
            mlp_infer_kernel<false, false><<<grid, 256, 0, st>>>(llr, llr_rows, ids, x, batch, w, wb, logits, order,
                                                                pin0);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

MlpWorkspace mlp_carve(void* base, int64_t batch)
{
    MlpWorkspace w;
    unsigned char* p = reinterpret_cast<unsigned char*>(base);
    int64_t o = 0;
    auto take = [&](int64_t bytes) { void* r = p ? p + o : nullptr; o += align256(bytes); return r; };
    // weight gradients reduce over the batch: enough splits to fill the device
    // (at least MLP_KCHUNK_MIN rows each, at most MLP_SPLITS_MAX of them)
    int64_t kchunk = (batch + MLP_SPLITS_MAX - 1) / MLP_SPLITS_MAX;
    kchunk = kchunk < MLP_KCHUNK_MIN ? MLP_KCHUNK_MIN : (kchunk + 31) / 32 * 32;
    const int splits = (int)((batch + kchunk - 1) / kchunk);
    w.h1 = (uint16_t*)take(batch * MLP_HID * 2);
    w.h2 = (uint16_t*)take(batch * MLP_HID * 2);
    w.logits = (float*)take(batch * MLP_OUT * 4);
    w.dl = (uint16_t*)take(batch * MLP_OUT * 2);
    w.dz2 = (uint16_t*)take(batch * MLP_HID * 2);
    w.dz1 = (uint16_t*)take(batch * MLP_HID * 2);
    // (room for the most splits any batch of this size or smaller uses, so the
    // work space grows with the batch)
    const int64_t room = (batch + MLP_KCHUNK_MIN - 1) / MLP_KCHUNK_MIN;
    w.part = (float*)take((room < MLP_SPLITS_MAX ? room : MLP_SPLITS_MAX) * MLP_HID * MLP_HID * 4);
    w.rowloss = (float*)take(batch * 4);
    w.splits = splits;
    w.kchunk = (int)kchunk;
    w.bytes = o;
    return w;
}

template <bool AK, bool BK, int EPI>
static void gemm(const uint16_t* A, int64_t a_i, int64_t a_k, const uint16_t* B, int64_t b_k, int64_t b_j, int M,
                 int N, int K, int splits, int kchunk, const float* bias, void* out, int64_t ldo,
                 const uint16_t* mask, int64_t ldm, hipStream_t st)
{
    dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
    gemm_kernel<AK, BK, EPI><<<grid, 256, 0, st>>>(A, a_i, a_k, B, b_k, b_j, M, N, K, kchunk, bias, out, ldo,
                                                   mask, ldm);
}

hipError_t mlp_features(const float* llr, int64_t batch, uint16_t* x, hipStream_t st, const int64_t* ids)
{
    if (batch > 0) features_kernel<<<(unsigned)((batch + 3) / 4), 256, 0, st>>>(llr, batch, x, ids);
    return hipGetLastError();
}

hipError_t mlp_prepare(const float* w, uint16_t* wb, uint16_t* wt, hipStream_t st)
{
    prepare_kernel<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(w, wb, wt);
    return hipGetLastError();
}

// Forward; activations h1, h2 kept in the work space (for the backward).
hipError_t mlp_forward(const float* w, const uint16_t* wb, const uint16_t* x, int64_t batch, float* logits,
                       const MlpWorkspace& ws, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    const int Bm = (int)batch;
    gemm<true, true, EPI_HIDDEN>(x, MLP_IN, 1, wb + MLP_OFF_W1, 1, MLP_IN, Bm, MLP_HID, MLP_IN, 1, MLP_IN,
                                 w + MLP_OFF_B1, ws.h1, MLP_HID, nullptr, 0, st);
    gemm<true, true, EPI_HIDDEN>(ws.h1, MLP_HID, 1, wb + MLP_OFF_W2, 1, MLP_HID, Bm, MLP_HID, MLP_HID, 1, MLP_HID,
                                 w + MLP_OFF_B2, ws.h2, MLP_HID, nullptr, 0, st);
    gemm<true, true, EPI_LOGITS>(ws.h2, MLP_HID, 1, wb + MLP_OFF_W3, 1, MLP_HID, Bm, MLP_OUT, MLP_HID, 1, MLP_HID,
                                 w + MLP_OFF_B3, logits, MLP_OUT, nullptr, 0, st);
    return hipGetLastError();
}

// Backward: forward, softmax cross-entropy, gradients of all parameters, mean loss.
hipError_t mlp_backward(const float* w, const uint16_t* wb, const uint16_t* wt, const uint16_t* x,
                        const int32_t* labels, int64_t batch, float* grads, float* loss, const MlpWorkspace& ws,
                        hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    hipError_t e = mlp_forward(w, wb, x, batch, ws.logits, ws, st);
    if (e != hipSuccess) return e;
    const int Bm = (int)batch;
    const int S = ws.splits, KC = ws.kchunk;
    softmax_ce_kernel<<<(unsigned)((batch + 3) / 4), 256, 0, st>>>(ws.logits, labels, batch, ws.dl, ws.rowloss);
    sum_kernel<<<1, 256, 0, st>>>(ws.rowloss, batch, 1.0f / (float)batch, loss);
    // layer 3: dW3 = dl^T h2, db3 = colsum(dl), dz2 = (dl W3) * [h2 > 0]
    gemm<false, false, EPI_PARTIAL>(ws.dl, 1, MLP_OUT, ws.h2, MLP_HID, 1, MLP_OUT, MLP_HID, Bm, S, KC, nullptr,
                                    ws.part, 0, nullptr, 0, st);
    reduce_partials_kernel<<<(MLP_OUT * MLP_HID + 255) / 256, 256, 0, st>>>(ws.part, S, MLP_OUT * MLP_HID,
                                                                           grads + MLP_OFF_W3);
    colsum_kernel<<<dim3(1, S), 256, 0, st>>>(ws.dl, batch, MLP_OUT, KC, ws.part);
    reduce_partials_kernel<<<1, 256, 0, st>>>(ws.part, S, MLP_OUT, grads + MLP_OFF_B3);
    gemm<true, true, EPI_MASKED>(ws.dl, MLP_OUT, 1, wt + MLP_T_W3, 1, MLP_OUT, Bm, MLP_HID, MLP_OUT, 1, MLP_OUT,
                                 nullptr, ws.dz2, MLP_HID, ws.h2, MLP_HID, st);
    // layer 2
    gemm<false, false, EPI_PARTIAL>(ws.dz2, 1, MLP_HID, ws.h1, MLP_HID, 1, MLP_HID, MLP_HID, Bm, S, KC,
                                    nullptr, ws.part, 0, nullptr, 0, st);
    reduce_partials_kernel<<<(MLP_HID * MLP_HID + 255) / 256, 256, 0, st>>>(ws.part, S, MLP_HID * MLP_HID,
                                                                           grads + MLP_OFF_W2);
    colsum_kernel<<<dim3(1, S), 256, 0, st>>>(ws.dz2, batch, MLP_HID, KC, ws.part);
    reduce_partials_kernel<<<1, 256, 0, st>>>(ws.part, S, MLP_HID, grads + MLP_OFF_B2);
    gemm<true, true, EPI_MASKED>(ws.dz2, MLP_HID, 1, wt + MLP_T_W2, 1, MLP_HID, Bm, MLP_HID, MLP_HID, 1, MLP_HID,
                                 nullptr, ws.dz1, MLP_HID, ws.h1, MLP_HID, st);
    // layer 1
    gemm<false, false, EPI_PARTIAL>(ws.dz1, 1, MLP_HID, x, MLP_IN, 1, MLP_HID, MLP_IN, Bm, S, KC, nullptr,
                                    ws.part, 0, nullptr, 0, st);
    reduce_partials_kernel<<<(MLP_HID * MLP_IN + 255) / 256, 256, 0, st>>>(ws.part, S, MLP_HID * MLP_IN,
                                                                          grads + MLP_OFF_W1);
    colsum_kernel<<<dim3(1, S), 256, 0, st>>>(ws.dz1, batch, MLP_HID, KC, ws.part);
    reduce_partials_kernel<<<1, 256, 0, st>>>(ws.part, S, MLP_HID, grads + MLP_OFF_B1);
    return hipGetLastError();
}

hipError_t mlp_adam(float* w, float* m, float* v, const float* g, float lr, int step, uint16_t* wb, uint16_t* wt,
                    hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    adam_kernel<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(w, m, v, g, lr, b1, b2, eps, c1, c2, wb, wt);
    return hipGetLastError();
}

hipError_t mlp_order(const float* logits, int64_t batch, uint8_t* order, hipStream_t st, bool pin0)
{
    if (batch > 0) order_kernel<<<(unsigned)((batch + 3) / 4), 256, 0, st>>>(logits, batch, order, pin0 ? 1 : 0);
    return hipGetLastError();
}

}  // namespace orbg
