// Decode kernels with 8 keys per lane (codes with n <= 512).
#include "decode_impl.h"

namespace orbg {
template hipError_t launch_decode_nk<8>(const DecodeArgs& a, bool s32, hipStream_t stream);
}  // namespace orbg
