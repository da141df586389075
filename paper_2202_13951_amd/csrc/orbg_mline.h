// Full (m-line) ORBGRAND kernel interface (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ORBG_ML_WMAX 22          // flips per pattern the order reaches within the budget limit
#define ORBG_ML_SMAX 4096        // partial logistic weights 0..4095 (the order reaches no larger one)
#define ORBG_ML_LMAX 512         // largest code length (and segment length)
#define ORBG_ML_MSEG 4           // largest number of segments
#define ORBG_ML_WINCAP 22        // flips of one pattern
#define ORBG_ML_BUDGET_MAX 5000000  // largest query budget
#define ORBG_ML_QCAP 64          // queued splits: fewer than 64 untested patterns plus one

namespace orbg {

struct MlineArgs {
    const float* llr;          // nblocks x n
    int n;
    int m;                     // n - k
    const uint64_t* cols;      // n packed parity-check columns
    const uint64_t* rows;      // m x nk packed rows (nk = 1, 2, 4, 8 for n <= 64, 128, 256, 512)
    int64_t nblocks;
    uint32_t budget;
    int mseg;                  // largest number of segments of the fit
    bool jdiv;                 // J_{i-1} rounded to a multiple of beta_i
    const uint32_t* table;     // subset counts, subset_table_words() entries
    uint8_t* cw;
    uint64_t* queries;
    uint8_t* abandoned;
    int32_t* mfit;             // per-block segment count, or nullptr
    int32_t* j0;               // per-block J_0 of the fit (the 1-line offset for one segment), or nullptr
};

// Entries of the subset-count table: (LMAX + 1) x (WMAX + 1) x SMAX.
constexpr size_t subset_table_words() { return (size_t)(ORBG_ML_LMAX + 1) * (ORBG_ML_WMAX + 1) * ORBG_ML_SMAX; }

hipError_t build_subset_table(uint32_t* t, hipStream_t stream);
hipError_t launch_mline(const MlineArgs& a, int grid, hipStream_t stream);
// The kernels for fits of at most MM segments (one translation unit each).
template <int MM>
hipError_t launch_mline_m(const MlineArgs& a, int grid, hipStream_t stream);
extern template hipError_t launch_mline_m<1>(const MlineArgs&, int, hipStream_t);
extern template hipError_t launch_mline_m<2>(const MlineArgs&, int, hipStream_t);
extern template hipError_t launch_mline_m<3>(const MlineArgs&, int, hipStream_t);
extern template hipError_t launch_mline_m<4>(const MlineArgs&, int, hipStream_t);

}  // namespace orbg
