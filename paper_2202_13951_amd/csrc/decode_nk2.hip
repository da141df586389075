// Decode kernels with 2 keys per lane (codes with n <= 128).
#include "decode_impl.h"

namespace orbg {
template hipError_t launch_decode_nk<2>(const DecodeArgs& a, bool s32, hipStream_t stream);
}  // namespace orbg
