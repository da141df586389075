// Sanitizer driver for the C-ABI front end (test infrastructure): calls every
// entry point of include/orbgrand.h with arguments its host-side checks must
// reject (and a few that pass them and then fail without a device), and checks
// the status and message.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize.py against capi.hip
// (host only) and the launcher stand-ins; exits 0 when every check holds.
#include <cstdio>
#include <cstring>
#include <vector>

#include "orbgrand.h"

static int fails = 0;
static void expect(int rc, int want, const char* part, int line)
{
    const char* msg = orbg_last_error();
    if (rc != want || (part && !std::strstr(msg, part))) {
        std::fprintf(stderr, "line %d: rc %d (want %d), message '%s' (want '%s')\n", line, rc, want, msg,
                     part ? part : "");
        ++fails;
    }
}
#define EXPECT(call, want, part) expect((call), (want), (part), __LINE__)

int main()
{
    std::vector<uint8_t> H(6 * 32, 0);
    for (int r = 0; r < 6; ++r) H[r * 32 + 26 + r] = 1;
    void* p = (void*)&H[0];                       // a non-null pointer, never dereferenced as a device buffer
    uint8_t* u8 = (uint8_t*)p;
    // code arguments
    EXPECT(orbg_decode(nullptr, (float*)p, 32, 26, 100, 4, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "H is NULL");
    EXPECT(orbg_decode(H.data(), (float*)p, 0, 0, 100, 4, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "n = 0");
    EXPECT(orbg_decode(H.data(), (float*)p, 1025, 1000, 100, 4, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "n = 1025");
    EXPECT(orbg_decode(H.data(), (float*)p, 32, 32, 100, 4, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "n - k");
    H[5] = 2;
    EXPECT(orbg_decode(H.data(), (float*)p, 32, 26, 100, 4, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "not 0 or 1");
    H[5] = 0;
    EXPECT(orbg_decode(H.data(), (float*)p, 32, 26, 0, 4, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "budget");
    EXPECT(orbg_decode(H.data(), (float*)p, 32, 26, 5000001, 4, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "budget");
    EXPECT(orbg_decode(H.data(), (float*)p, 32, 26, 100, -1, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "negative");
    EXPECT(orbg_decode(H.data(), nullptr, 32, 26, 100, 4, u8, (uint64_t*)p, u8, nullptr), ORBG_EINVAL, "NULL");
    // past the checks: no device here, so the first device call fails
    {
        const int rc = orbg_decode(H.data(), (float*)p, 32, 26, 100, 4, u8, (uint64_t*)p, u8, nullptr);
        if (rc >= 0) { std::fprintf(stderr, "decode without a device returned %d\n", rc); ++fails; }
    }
    EXPECT(orbg_decode_ordered(H.data(), (float*)p, 32, 26, 100, 4, nullptr, u8, (uint64_t*)p, u8, nullptr),
           ORBG_EINVAL, "order");
    orbg_launch_params lp = {};
    lp.workgroups_per_cu = 65;
    EXPECT(orbg_decode_ex(H.data(), (float*)p, 32, 26, 100, 4, nullptr, u8, (uint64_t*)p, u8, &lp, nullptr),
           ORBG_EINVAL, "workgroups_per_cu");
    lp = orbg_launch_params{};
    lp.one_block_per_workgroup = 2;
    EXPECT(orbg_decode_ex(H.data(), (float*)p, 32, 26, 100, 4, nullptr, u8, (uint64_t*)p, u8, &lp, nullptr),
           ORBG_EINVAL, "one_block_per_workgroup");
    EXPECT(orbg_decode_1line(H.data(), (float*)p, 32, 26, 5000001, 4, u8, (uint64_t*)p, u8, nullptr, nullptr,
                             nullptr),
           ORBG_EINVAL, "budget");
    {
        // past the 1-line schedules' budget limit and past the m-line kernel's length
        std::vector<uint8_t> H600(10 * 600, 0);
        EXPECT(orbg_decode_1line(H600.data(), (float*)p, 600, 590, (1u << 22) + 1, 4, u8, (uint64_t*)p, u8, nullptr,
                                 nullptr, nullptr),
               ORBG_EINVAL, "above 2^22");
    }
    EXPECT(orbg_decode_mline(H.data(), (float*)p, 32, 26, 100, 4, 5, 0, u8, (uint64_t*)p, u8, nullptr, nullptr),
           ORBG_EINVAL, "segments");
    EXPECT(orbg_decode_mline(H.data(), (float*)p, 32, 26, 100, 4, 2, 2, u8, (uint64_t*)p, u8, nullptr, nullptr),
           ORBG_EINVAL, "jdiv");
    // registry and mixed decodes
    int id = -1;
    EXPECT(orbg_code_register(H.data(), 32, 26, nullptr), ORBG_EINVAL, "code_id is NULL");
    EXPECT(orbg_code_release(12345), ORBG_EINVAL, "not registered");
    const int ids[1] = {77};
    EXPECT(orbg_decode_mixed(ids, 1, u8, (int64_t*)p, (float*)p, -1, 4, 100, u8, 10, (uint64_t*)p, u8, nullptr,
                             nullptr),
           ORBG_EINVAL, "must not be negative");
    EXPECT(orbg_decode_mixed(ids, 9, u8, (int64_t*)p, (float*)p, 10, 4, 100, u8, 10, (uint64_t*)p, u8, nullptr,
                             nullptr),
           ORBG_EINVAL, "ncodes");
    EXPECT(orbg_decode_mixed(ids, 1, u8, (int64_t*)p, (float*)p, 10, 4, 100, u8, 10, (uint64_t*)p, u8, nullptr,
                             nullptr),
           ORBG_EINVAL, "not registered");
    EXPECT(orbg_decode_mixed_noalloc(ids, 1, u8, (int64_t*)p, (float*)p, 10, ORBG_NOALLOC_BATCH_MAX + 1, 100, u8, 10,
                                     (uint64_t*)p, u8, nullptr, nullptr),
           ORBG_EINVAL, "above");
    (void)id;
    // schedules
    std::vector<uint8_t> out(16 * 8);
    EXPECT(orbg_schedule_export(0, 8, out.data(), nullptr), ORBG_EINVAL, "n = 0");
    EXPECT(orbg_schedule_export(32, 0, out.data(), nullptr), ORBG_EINVAL, "count");
    EXPECT(orbg_schedule_export(32, 8, nullptr, nullptr), ORBG_EINVAL, "out is NULL");
    int j0max = 0;
    EXPECT(orbg_schedule_export_1line(32, 100, -2, 8, out.data(), &j0max, nullptr), ORBG_EINVAL, "j0 = -2");
    EXPECT(orbg_schedule_export_1line(32, 100, 0, 101, out.data(), &j0max, nullptr), ORBG_EINVAL, "above the budget");
    // network
    if (orbg_mlp_workspace_bytes(-1) != -1) { std::fprintf(stderr, "workspace bytes of -1\n"); ++fails; }
    EXPECT(orbg_mlp_features((float*)p, 127, 4, (uint16_t*)p, nullptr), ORBG_EINVAL, "n = 128");
    EXPECT(orbg_mlp_forward((float*)p, (uint16_t*)p, (uint16_t*)p, 4, (float*)p, p, 1, nullptr), ORBG_EINVAL,
           "smaller");
    EXPECT(orbg_mlp_backward((float*)p, (uint16_t*)p, (uint16_t*)p, (uint16_t*)p, (int32_t*)p, 0, (float*)p,
                             (float*)p, p, 1 << 20, nullptr),
           ORBG_EINVAL, "batch >= 1");
    EXPECT(orbg_mlp_adam((float*)p, (float*)p, (float*)p, (float*)p, 2.0f, 1, (uint16_t*)p, (uint16_t*)p, nullptr),
           ORBG_EINVAL, "lr");
    EXPECT(orbg_mlp_adam((float*)p, (float*)p, (float*)p, (float*)p, 0.1f, 0, (uint16_t*)p, (uint16_t*)p, nullptr),
           ORBG_EINVAL, "step");
    EXPECT(orbg_mlp_order(nullptr, 4, u8, nullptr), ORBG_EINVAL, "NULL");
    EXPECT(orbg_mlp_infer((float*)p, (uint16_t*)p, (float*)p, 4, nullptr, nullptr, -1, (float*)p, nullptr, 0,
                          nullptr),
           ORBG_EINVAL, "batch");
    EXPECT(orbg_mlp_infer((float*)p, (uint16_t*)p, (float*)p, 4, nullptr, nullptr, 4, nullptr, nullptr, 0, nullptr),
           ORBG_EINVAL, "no output");
    EXPECT(orbg_mlp_infer((float*)p, (uint16_t*)p, nullptr, 4, nullptr, nullptr, 4, (float*)p, nullptr, 0, nullptr),
           ORBG_EINVAL, "NULL");
    EXPECT(orbg_mlp_infer((float*)p, (uint16_t*)p, (float*)p, -3, nullptr, nullptr, 4, (float*)p, nullptr, 0, nullptr),
           ORBG_EINVAL, "llr_rows");
    EXPECT(orbg_mlp_infer((float*)p, (uint16_t*)p, (float*)p, 4, nullptr, nullptr, 4, (float*)p, u8, 2, nullptr),
           ORBG_EINVAL, "pin0");
    EXPECT(orbg_mlp_infer((float*)p, (uint16_t*)p, (float*)p, 4, nullptr, nullptr, 4, (float*)p, u8, 1, nullptr),
           ORBG_EHIP, "inference launch failed");
    if (orbg_learned_workspace_bytes(-1) != -1) { std::fprintf(stderr, "learned workspace bytes of -1\n"); ++fails; }
    std::vector<uint8_t> H128(23 * 128, 0);
    for (int r = 0; r < 23; ++r) H128[r * 128 + 105 + r] = 1;
    EXPECT(orbg_decode_learned(H.data(), (float*)p, 32, 26, 100, 4, (float*)p, (uint16_t*)p, p, 1 << 30, u8,
                               (uint64_t*)p, u8, nullptr, nullptr, nullptr, nullptr),
           ORBG_EINVAL, "n = 128");
    EXPECT(orbg_decode_learned(H128.data(), (float*)p, 128, 105, 100, 4, (float*)p, (uint16_t*)p, p, 1, u8,
                               (uint64_t*)p, u8, nullptr, nullptr, nullptr, nullptr),
           ORBG_EINVAL, "smaller");
    if (fails) { std::fprintf(stderr, "%d checks failed\n", fails); return 1; }
    std::printf("C-ABI sanitizer driver: all checks passed\n");
    return 0;
}
