// Decode kernels with 1 key per lane (codes with n <= 64).
#include "decode_impl.h"

namespace orbg {
template hipError_t launch_decode_nk<1>(const DecodeArgs& a, bool s32, hipStream_t stream);
}  // namespace orbg
