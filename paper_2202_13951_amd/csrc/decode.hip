// Dispatch of a decode to the kernels of its keys per lane (decode_nk*.hip);
// the kernels themselves are in decode_impl.h.
#include "orbg_kernels.h"

namespace orbg {

template <int NKMAX>
hipError_t launch_decode_nk(const DecodeArgs& a, bool s32, hipStream_t stream);
extern template hipError_t launch_decode_nk<1>(const DecodeArgs&, bool, hipStream_t);
extern template hipError_t launch_decode_nk<2>(const DecodeArgs&, bool, hipStream_t);
extern template hipError_t launch_decode_nk<4>(const DecodeArgs&, bool, hipStream_t);
extern template hipError_t launch_decode_nk<8>(const DecodeArgs&, bool, hipStream_t);
extern template hipError_t launch_decode_nk<16>(const DecodeArgs&, bool, hipStream_t);

hipError_t launch_decode(const DecodeArgs& a, hipStream_t stream)
{
    if (a.nblocks < 1) return hipSuccess;
    int nk = 1, mmax = 0;
    for (int i = 0; i < a.codes.ncodes; ++i) {
        nk = a.codes.c[i].nk > nk ? a.codes.c[i].nk : nk;
        mmax = a.codes.c[i].m > mmax ? a.codes.c[i].m : mmax;
    }
    const bool s32 = mmax <= 32;
    if (a.oneline && (a.mixed || a.order)) return hipErrorInvalidValue;   // one code, plain batch order
    if (a.mixed && nk > 4) return hipErrorInvalidValue;                  // mixed launches take n <= 256
    if (nk <= 1) return launch_decode_nk<1>(a, s32, stream);
    if (nk <= 2) return launch_decode_nk<2>(a, s32, stream);
    if (nk <= 4) return launch_decode_nk<4>(a, s32, stream);
    if (nk <= 8) return launch_decode_nk<8>(a, s32, stream);
    return launch_decode_nk<16>(a, s32, stream);
}

}  // namespace orbg
