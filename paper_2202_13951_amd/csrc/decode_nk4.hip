// Decode kernels with 4 keys per lane (codes with n <= 256).
#include "decode_impl.h"

namespace orbg {
template hipError_t launch_decode_nk<4>(const DecodeArgs& a, bool s32, hipStream_t stream);
}  // namespace orbg
