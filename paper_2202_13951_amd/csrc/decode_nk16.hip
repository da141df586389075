// Decode kernels with 16 keys per lane (codes with n <= 1024).
#include "decode_impl.h"

namespace orbg {
template hipError_t launch_decode_nk<16>(const DecodeArgs& a, bool s32, hipStream_t stream);
}  // namespace orbg
