// Kernel launchers of liborbgrand (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace orbg {

struct DecodeArgs {
    const float* llr;          // device, nblocks x n
    int64_t nblocks;
    int n;
    int m;                     // n - k
    const uint64_t* cols;      // device, n packed parity-check columns
    const uint2* sched;        // device schedule entries (packed, see Schedule)
    const uint32_t* bh;        // device per-batch count of ranks above 8
    uint64_t slen;             // schedule entries
    int rdepth;                // ranks whose columns are staged (<= 255)
    uint64_t budget;
    const uint8_t* order;      // device, nblocks x 64, or nullptr for plain order
    uint8_t* cw;               // device, nblocks x n
    uint64_t* queries;         // device, nblocks
    uint8_t* abandoned;        // device, nblocks
    int64_t max_workgroups;    // cap on the persistent grid (0 = no cap)
    unsigned long long* work;  // device work counter (reset by the launch)
    int chunk;                 // blocks taken per counter increment
};

hipError_t launch_decode(const DecodeArgs& a, hipStream_t stream);

}  // namespace orbg
