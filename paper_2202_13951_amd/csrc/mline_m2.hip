// Full (m-line) ORBGRAND decode kernels for fits of at most 2 segments.
#include "mline_impl.h"

namespace orbg {
template hipError_t launch_mline_m<2>(const MlineArgs& a, int grid, hipStream_t stream);
}  // namespace orbg
