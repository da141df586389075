// Full (m-line) ORBGRAND decode (Sec. III-D; fit of Sec. III-E): the device
// table of subset counts the unranking reads, and the launch, which picks the
// kernel compiled for the request's largest segment count (mline_impl.h).
#include "orbg_device.h"
#include "orbg_internal.h"
#include "orbg_mline.h"

namespace orbg {

namespace {

constexpr int WL = ORBG_ML_WMAX;          // partial Hamming weights 0..22
constexpr int SL = ORBG_ML_SMAX;          // partial logistic weights 0..4095

// One step of the subset-count recursion: table for `len` from the one for len - 1.
__global__ void __launch_bounds__(256) subset_table_step(uint32_t* t, int len)
{
    const int cells = (WL + 1) * SL;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    uint32_t* cur = t + (size_t)len * cells;
    if (len == 0) {
        cur[c] = c == 0 ? 1u : 0u;
        return;
    }
    const uint32_t* prev = t + (size_t)(len - 1) * cells;
    const int w = c / SL, s = c % SL;
    uint64_t v = prev[c];
    if (w >= 1 && s >= len) v += prev[(w - 1) * SL + (s - len)];
    cur[c] = v > 0xffffffffull ? 0xffffffffu : (uint32_t)v;
}

}  // namespace

hipError_t build_subset_table(uint32_t* t, hipStream_t stream)
{
    const int cells = (WL + 1) * SL;
    for (int len = 0; len <= ORBG_ML_LMAX; ++len) {
        subset_table_step<<<(cells + 255) / 256, 256, 0, stream>>>(t, len);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_mline(const MlineArgs& a, int grid, hipStream_t stream)
{
    if (a.nblocks <= 0) return hipSuccess;
    switch (a.mseg) {
    case 1: return launch_mline_m<1>(a, grid, stream);
    case 2: return launch_mline_m<2>(a, grid, stream);
    case 3: return launch_mline_m<3>(a, grid, stream);
    default: return launch_mline_m<4>(a, grid, stream);
    }
}

}  // namespace orbg
