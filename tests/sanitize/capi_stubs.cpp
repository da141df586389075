// Stand-ins for the device-side launchers of liborbgrand (test
// infrastructure): the sanitizer build of the C-ABI front end (capi.hip,
// compiled for the host only) links against these, so its argument checks,
// caches and error paths run under AddressSanitizer and
// UndefinedBehaviorSanitizer without a GPU.  Every launcher reports failure.
#include <hip/hip_runtime.h>

#include "orbg_internal.h"
#include "orbg_kernels.h"
#include "orbg_mline.h"
#include "orbg_mlp.h"

namespace orbg {

hipError_t launch_decode(const DecodeArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_mline(const MlineArgs&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t build_subset_table(uint32_t*, hipStream_t) { return hipErrorNotSupported; }
int orbg_build_schedule(int, uint64_t, hipStream_t, Schedule*, char* err, size_t errlen)
{
    snprintf(err, errlen, "no device in the sanitizer build");
    return -3;
}
int orbg_build_schedule_1line(int, uint64_t, hipStream_t, Schedule1*, char* err, size_t errlen)
{
    snprintf(err, errlen, "no device in the sanitizer build");
    return -3;
}
int orbg_unpack_entries(const uint2*, uint64_t, uint8_t*, hipStream_t) { return -3; }
int orbg_unpack_schedule(const Schedule*, uint64_t, uint8_t*, hipStream_t) { return -3; }
MlpWorkspace mlp_carve(void*, int64_t batch)
{
    MlpWorkspace w = {};
    w.bytes = batch * 4096;
    return w;
}
hipError_t mlp_features(const float*, int64_t, uint16_t*, hipStream_t, const int64_t*) { return hipErrorNotSupported; }
hipError_t mlp_prepare(const float*, uint16_t*, uint16_t*, hipStream_t) { return hipErrorNotSupported; }
hipError_t mlp_forward(const float*, const uint16_t*, const uint16_t*, int64_t, float*, const MlpWorkspace&,
                       hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t mlp_backward(const float*, const uint16_t*, const uint16_t*, const uint16_t*, const int32_t*, int64_t,
                        float*, float*, const MlpWorkspace&, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t mlp_adam(float*, float*, float*, const float*, float, int, uint16_t*, uint16_t*, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t mlp_order(const float*, int64_t, uint8_t*, hipStream_t, bool) { return hipErrorNotSupported; }
hipError_t mlp_order_table(const uint8_t*, const int64_t*, int64_t, int64_t, uint8_t*, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t mlp_infer(const float*, const uint16_t*, const float*, int64_t, const int64_t*, const uint16_t*, int64_t,
                     float*, uint8_t*, bool, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace orbg
