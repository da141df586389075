// Host/device shared internals of liborbgrand (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#define ORBG_WCAP 255        // subset-sum counts are kept for logistic weights 0..255
#define ORBG_WMAX_H 16       // largest Hamming weight a schedule entry holds
#define ORBG_WLEVEL_MAX 152  // every pattern of logistic weight <= 152 has at most 16 flips
#define ORBG_NMAX 1024       // largest code length
#define ORBG_MMAX 64         // largest redundancy n - k (syndromes are one u64)
#define ORBG_BUDGET_MAX (1ull << 28)

namespace orbg {

struct ClassInfo {
    int W;
    int w;
    uint64_t offset;
    uint64_t count;
};

// Device-resident query schedule for one (n, len).
struct Schedule {
    int n;
    uint64_t len;       // number of valid entries
    uint4* entries;     // nbatch * 64 entries of 16 u8 ranks (1-based, 0 = none)
    uint8_t* bw;        // per batch of 64: largest number of ranks in an entry
    uint64_t nbatch;
    int rmax;           // largest rank any entry references
    int wlast;          // logistic weight of the last entry
};

int orbg_build_schedule(int n, uint64_t len, hipStream_t stream, Schedule* out, char* err, size_t errlen);

}  // namespace orbg
