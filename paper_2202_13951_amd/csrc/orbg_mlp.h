// Learned-proposal network: sizes, parameter layout, launchers (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MLP_IN 128
#define MLP_HID 256
#define MLP_OUT 64
// flat FP32 / BF16 parameter layout (output x input, row-major)
#define MLP_OFF_W1 0
#define MLP_OFF_B1 (MLP_OFF_W1 + MLP_HID * MLP_IN)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_HID)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_HID * MLP_HID)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_HID)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_OUT * MLP_HID)
#define MLP_NPARAM (MLP_OFF_B3 + MLP_OUT)
// transposed BF16 weight copies (input x output)
#define MLP_T_W1 0
#define MLP_T_W2 (MLP_T_W1 + MLP_IN * MLP_HID)
#define MLP_T_W3 (MLP_T_W2 + MLP_HID * MLP_HID)
#define MLP_NTRANS (MLP_T_W3 + MLP_HID * MLP_OUT)
#define MLP_KCHUNK_MIN 256   // fewest batch rows per split of a weight-gradient GEMM
#define MLP_SPLITS_MAX 64    // most splits of a weight-gradient GEMM
#define MLP_BATCH_MAX (1 << 20)

namespace orbg {

struct MlpWorkspace {
    uint16_t* h1;
    uint16_t* h2;
    float* logits;
    uint16_t* dl;
    uint16_t* dz2;
    uint16_t* dz1;
    float* part;
    float* rowloss;
    int splits;              // batch rows split into `splits` chunks of `kchunk` (a multiple of 32)
    int kchunk;
    int64_t bytes;
};

// Carves the work space of a `batch`-row call out of `base` (base may be
// nullptr to only compute .bytes).
MlpWorkspace mlp_carve(void* base, int64_t batch);

hipError_t mlp_features(const float* llr, int64_t batch, uint16_t* x, hipStream_t st, const int64_t* ids = nullptr);
hipError_t mlp_prepare(const float* w, uint16_t* wb, uint16_t* wt, hipStream_t st);
hipError_t mlp_forward(const float* w, const uint16_t* wb, const uint16_t* x, int64_t batch, float* logits,
                       const MlpWorkspace& ws, hipStream_t st);
hipError_t mlp_backward(const float* w, const uint16_t* wb, const uint16_t* wt, const uint16_t* x,
                        const int32_t* labels, int64_t batch, float* grads, float* loss, const MlpWorkspace& ws,
                        hipStream_t st);
hipError_t mlp_adam(float* w, float* m, float* v, const float* g, float lr, int step, uint16_t* wb, uint16_t* wt,
                    hipStream_t st);
hipError_t mlp_order(const float* logits, int64_t batch, uint8_t* order, hipStream_t st, bool pin0 = false);
// Fused inference without a work space: features of llr rows (ids[b], or b;
// rows outside [0, llr_rows) read as zeros) or the given features x (llr ==
// nullptr), the three layers, and the logits and/or the batch order (either may
// be nullptr, not both).
hipError_t mlp_infer(const float* w, const uint16_t* wb, const float* llr, int64_t llr_rows, const int64_t* ids,
                     const uint16_t* x, int64_t batch, float* logits, uint8_t* order, bool pin0, hipStream_t st);
hipError_t mlp_order_table(const uint8_t* rows, const int64_t* ids, int64_t count, int64_t batch, uint8_t* order,
                           hipStream_t st);

}  // namespace orbg
