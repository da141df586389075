// Host/device shared internals of liborbgrand (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#define ORBG_WCAP 255        // subset-sum counts are kept for logistic weights 0..255
#define ORBG_WMAX_H 16       // largest Hamming weight a schedule entry holds
#define ORBG_WLEVEL_MAX 152  // every pattern of logistic weight <= 152 has at most 16 flips
#define ORBG_NMAX 1024       // largest code length
#define ORBG_XCDS 8          // accelerator complex dies per MI355X (workgroups dealt round-robin)
#define ORBG_COUNTER_STRIDE 32  // u64 stride between work counters (256 B apart)
#define ORBG_MMAX 64         // largest redundancy n - k (syndromes are one u64)
#define ORBG_BUDGET_MAX 5000000ull    // the abandonment threshold the paper uses (Sec. IV-A)
#define ORBG_BUDGET_MAX_1LINE (1ull << 22)
#define ORBG_SCHED_POW2_MAX (1ull << 22)  // schedules up to this length are rounded up to a power of two
#define ORBG_LOW_RANKS 8     // ranks 1..8 are flipped through a per-block subset table
#define ORBG_HIGH_SLOTS 7    // ranks above 8 held by one entry (bytes 1..7)
#define ORBG_WLEVEL_PACKED 99  // every pattern of logistic weight <= 99 has at most 7 ranks above 8
#define ORBG_WLEVEL_SCHED 100  // the schedule also takes logistic weight 100 up to its one pattern
                               // with 8 ranks above 8, {9, ..., 16}, the last of its (W, w) class
#define ORBG_SCHED_PAD 6        // zero batches after a schedule's last batch

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
    uint2* entries;     // nbatch * 64 packed entries: byte 0 = mask of ranks 1..8 (bit j = rank j+1),
                        // bytes 1..7 = ranks above 8, ascending, 0 = none
    uint64_t nbatch;
    int rmax;           // largest rank any entry references
    int rmax0;          // largest rank an entry of the first batch of 64 references
    int wlast;          // logistic weight of the last entry
};

// 1-line ORBGRAND schedules for one (n, len): j0max + 2 schedules of `len`
// entries (same packing), the one for offset J0 at entries + (J0 + 1) * stride,
// J0 = -1 .. j0max; fitted offsets above j0max use the last one.
struct Schedule1 {
    int n;
    uint64_t len;
    uint64_t nbatch;    // batches of 64 per schedule
    uint64_t stride;    // entries per schedule including ORBG_SCHED_PAD zero batches
    int j0max;
    uint2* entries;
    int rmax;           // largest rank any schedule references
};

int orbg_build_schedule(int n, uint64_t len, hipStream_t stream, Schedule* out, char* err, size_t errlen);
int orbg_build_schedule_1line(int n, uint64_t len, hipStream_t stream, Schedule1* out, char* err, size_t errlen);
// Unpacks `count` entries from `entries` to 16-byte lists of 1-based ranks.
int orbg_unpack_entries(const uint2* entries, uint64_t count, uint8_t* d_out, hipStream_t stream);
// Unpacks the first `count` entries to 16-byte lists of 1-based ranks.
int orbg_unpack_schedule(const Schedule* s, uint64_t count, uint8_t* d_out, hipStream_t stream);

}  // namespace orbg
