// Kernel launchers of liborbgrand (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ORBG_MAX_CODES 8       // codes one launch may mix
#define ORBG_MIXED_COLS 2048   // packed columns of all codes of a mixed launch (sum of n)

namespace orbg {

// One code of a launch (device pointers into the library's caches).
struct CodeDesc {
    int n;                     // code length
    int m;                     // n - k
    int nk;                    // keys per lane of the rank sort: power of two >= n / 64
    int rdepth;                // ranks whose columns are staged (<= 255)
    int rdepth0;               // ranks the first batch of 64 entries reaches
    uint32_t slen;             // schedule entries
    uint32_t col_base;         // first column of this code in the launch's LDS column table
    uint32_t row_base;         // first word of this code's rows in the launch's LDS row table
    const uint64_t* cols;      // n packed parity-check columns
    const uint64_t* rows;      // m x nk packed parity-check rows (bit l of word j = H[r][64 j + l])
    const uint2* sched;        // schedule entries for this n (1-line: the schedule of offset -1)
    int j0max;                 // 1-line: largest offset with a schedule of its own
    uint32_t sstride;          // 1-line: entries between the schedules of consecutive offsets
};

struct CodeTable {
    int ncodes;
    int rwords;                // row words of all codes (LDS row table size)
    CodeDesc c[ORBG_MAX_CODES];
};

// Launch shape (the autotuner's knobs).
struct LaunchParams {
    int wg_per_cu;             // light pass: one-wave workgroups per compute unit
    int chunk;                 // blocks per work-counter increment (0 = about 16 per wave)
    int split_steps;           // light pass stops a block after this many 64-query steps (0 = never)
    int heavy_waves;           // waves that share one heavy block (4, 8 or 16)
    int heavy_wg_per_cu;       // heavy pass: workgroups per compute unit
    int naive;                 // 1: one one-wave workgroup per block, no work counter, no heavy pass
};

struct DecodeArgs {
    CodeTable codes;
    bool mixed;                // per-block code index and row offsets given
    const uint8_t* block_code; // device, nblocks (mixed)
    const int64_t* row_off;    // device, nblocks: element offset of the row in llr and codeword (mixed)
    int64_t row_limit;         // mixed: rows must end within this many elements of llr and codeword
    const float* llr;
    int64_t nblocks;
    uint32_t budget;
    const uint8_t* order;      // device, nblocks x 64, or nullptr for plain order
    bool oneline;              // 1-line ORBGRAND order (one code, plain batch order)
    int32_t* j0;               // device, nblocks 1-line offsets, or nullptr
    uint8_t* cw;
    uint64_t* queries;
    uint8_t* abandoned;
    unsigned long long* ctrs;  // device work counters (8 slices, heavy count, heavy next)
    int64_t* heavy;            // device heavy-block list, capacity >= nblocks when splitting
    bool list_only;            // blocks left after split_steps are only listed in heavy (no heavy pass)
    const int64_t* ids;        // device, nblocks: caller's block index of each position, or nullptr
                               // (one code, no heavy pass; the batch order stays per position)
    bool skip0;                // ordered decode of blocks known to hold no member in batch 0:
                               // the search starts at step 1
    int cus;                   // compute units of the device
    LaunchParams p;
};

// Work slices of the light pass (8 per XCD), their stripe length in chunks, and
// the counter slots (u64 index, each on its own 128-byte line).
#define ORBG_SLICES 64
#define ORBG_STRIPE 64
#define ORBG_CTR_SLICE(x) ((x) * 16)
#define ORBG_CTR_HEAVY_COUNT (ORBG_SLICES * 16)
#define ORBG_CTR_HEAVY_NEXT ((ORBG_SLICES + 1) * 16)
#define ORBG_CTR_WORDS ((ORBG_SLICES + 2) * 16)

hipError_t launch_decode(const DecodeArgs& a, hipStream_t stream);

}  // namespace orbg
