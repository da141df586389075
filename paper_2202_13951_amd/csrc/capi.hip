// C-ABI front end of liborbgrand: argument checks, device caches of packed
// parity-check columns and query schedules, kernel launches.
#include "orbgrand.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "orbg_internal.h"
#include "orbg_kernels.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct CodeEntry {
    int n = 0, k = 0;
    std::vector<uint8_t> H;     // host copy, for exact cache matching
    uint64_t* d_cols = nullptr;
};

std::mutex g_mu;
// (device, hash) -> codes with that hash
std::map<std::pair<int, uint64_t>, std::vector<CodeEntry*>> g_codes;
// (device, n, len) -> schedule
std::map<std::tuple<int, int, uint64_t>, orbg::Schedule*> g_sched;
// (device, stream) -> work counter of the persistent decode grid
std::map<std::pair<int, hipStream_t>, unsigned long long*> g_work;
// device -> compute units
std::map<int, int> g_cus;

uint64_t fnv1a(const uint8_t* p, size_t len, uint64_t h = 1469598103934665603ull)
{
    for (size_t i = 0; i < len; ++i) { h ^= p[i]; h *= 1099511628211ull; }
    return h;
}

int check_code_args(const uint8_t* H, int n, int k)
{
    if (!H) return fail(ORBG_EINVAL, "H is NULL");
    if (n < 1 || n > ORBG_NMAX) return fail(ORBG_EINVAL, "n = %d outside [1, %d]", n, ORBG_NMAX);
    if (n - k < 1 || n - k > ORBG_MMAX || k < 0)
        return fail(ORBG_EINVAL, "n - k = %d outside [1, %d]", n - k, ORBG_MMAX);
    const size_t sz = (size_t)(n - k) * n;
    for (size_t i = 0; i < sz; ++i)
        if (H[i] > 1) return fail(ORBG_EINVAL, "H[%zu] = %u is not 0 or 1", i, (unsigned)H[i]);
    return ORBG_OK;
}

// Packed columns of H on the current device (cached by contents).
int get_code(const uint8_t* H, int n, int k, const uint64_t** cols)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ORBG_EHIP, "hipGetDevice failed");
    const size_t sz = (size_t)(n - k) * n;
    uint64_t h = fnv1a(H, sz);
    h = fnv1a(reinterpret_cast<const uint8_t*>(&n), sizeof(n), h);
    h = fnv1a(reinterpret_cast<const uint8_t*>(&k), sizeof(k), h);
    std::lock_guard<std::mutex> lk(g_mu);
    auto& bucket = g_codes[{dev, h}];
    for (CodeEntry* c : bucket)
        if (c->n == n && c->k == k && std::memcmp(c->H.data(), H, sz) == 0) { *cols = c->d_cols; return ORBG_OK; }
    std::vector<uint64_t> packed(n, 0ull);
    for (int r = 0; r < n - k; ++r)
        for (int i = 0; i < n; ++i)
            if (H[(size_t)r * n + i]) packed[i] |= 1ull << r;
    CodeEntry* c = new CodeEntry;
    c->n = n; c->k = k;
    c->H.assign(H, H + sz);
    if (hipMalloc(&c->d_cols, sizeof(uint64_t) * n) != hipSuccess) {
        delete c;
        return fail(ORBG_ENOMEM, "cannot allocate %d packed columns", n);
    }
    if (hipMemcpy(c->d_cols, packed.data(), sizeof(uint64_t) * n, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->d_cols);
        delete c;
        return fail(ORBG_EHIP, "copy of packed columns failed");
    }
    bucket.push_back(c);
    *cols = c->d_cols;
    return ORBG_OK;
}

uint64_t round_up_pow2(uint64_t x)
{
    uint64_t p = 64;
    while (p < x) p <<= 1;
    return p;
}

// Schedule with at least `need` entries for length n (need <= 2^n).
int get_schedule(int n, uint64_t need, hipStream_t stream, const orbg::Schedule** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ORBG_EHIP, "hipGetDevice failed");
    uint64_t len = round_up_pow2(need);
    if (n < 63 && len > (1ull << n)) len = 1ull << n;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(dev, n, len);
    auto it = g_sched.find(key);
    if (it != g_sched.end()) { *out = it->second; return ORBG_OK; }
    orbg::Schedule* s = new orbg::Schedule;
    char err[256] = {0};
    const int rc = orbg_build_schedule(n, len, stream, s, err, sizeof(err));
    if (rc != 0) {
        delete s;
        return fail(rc == -2 ? ORBG_ENOMEM : (rc == -1 ? ORBG_EINVAL : ORBG_EHIP), "%s", err);
    }
    g_sched[key] = s;
    *out = s;
    return ORBG_OK;
}

// Per-stream work counter (calls on one stream are ordered, so they can share it).
int get_work_counter(hipStream_t st, unsigned long long** out, int* cus)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ORBG_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_work.find({dev, st});
    if (it == g_work.end()) {
        unsigned long long* p = nullptr;
        if (hipMalloc(&p, 8 * ORBG_XCDS * ORBG_COUNTER_STRIDE) != hipSuccess)
            return fail(ORBG_ENOMEM, "cannot allocate work counters");
        it = g_work.emplace(std::make_pair(dev, st), p).first;
    }
    *out = it->second;
    auto c = g_cus.find(dev);
    if (c == g_cus.end()) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1) v = 256;
        c = g_cus.emplace(dev, v).first;
    }
    *cus = c->second;
    return ORBG_OK;
}

int decode_common(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                  const uint8_t* order, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned,
                  void* stream)
{
    int rc = check_code_args(H, n, k);
    if (rc) return rc;
    if (budget < 1 || budget > ORBG_BUDGET_MAX)
        return fail(ORBG_EINVAL, "budget = %llu outside [1, 2^22]", (unsigned long long)budget);
    if (batch < 0) return fail(ORBG_EINVAL, "batch = %lld is negative", (long long)batch);
    if (batch > 0 && (!llr || !codeword || !queries || !abandoned))
        return fail(ORBG_EINVAL, "a device buffer is NULL");
    if (order && n < 12) return fail(ORBG_EINVAL, "a batch order needs n >= 12 (got %d)", n);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const uint64_t* cols = nullptr;
    if ((rc = get_code(H, n, k, &cols))) return rc;
    uint64_t need = budget;
    if (order && need < 4096) need = 4096;
    if (n < 63 && need > (1ull << n)) need = 1ull << n;
    const orbg::Schedule* s = nullptr;
    if ((rc = get_schedule(n, need, st, &s))) return rc;
    if (batch == 0) return ORBG_OK;
    unsigned long long* work = nullptr;
    int cus = 0;
    if ((rc = get_work_counter(st, &work, &cus))) return rc;
    orbg::DecodeArgs a;
    a.llr = llr;
    a.nblocks = batch;
    a.n = n;
    a.m = n - k;
    a.cols = cols;
    a.sched = s->entries;
    a.bh = s->bh;
    a.slen = s->len;
    a.rdepth = s->rmax < n ? s->rmax : n;
    a.budget = budget;
    a.order = order;
    a.cw = codeword;
    a.queries = queries;
    a.abandoned = abandoned;
    a.max_workgroups = (int64_t)cus * 32;
    a.work = work;
    a.chunk = 0;
    const hipError_t e = orbg::launch_decode(a, st);
    if (e != hipSuccess) return fail(ORBG_EHIP, "decode launch failed: %s", hipGetErrorString(e));
    return ORBG_OK;
}

}  // namespace

extern "C" {

int orbg_decode(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                uint8_t* codeword, uint64_t* queries, uint8_t* abandoned, void* stream)
{
    g_err.clear();
    return decode_common(H, llr, n, k, budget, batch, nullptr, codeword, queries, abandoned, stream);
}

int orbg_decode_ordered(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                        const uint8_t* order, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned,
                        void* stream)
{
    g_err.clear();
    if (!order && batch > 0) return fail(ORBG_EINVAL, "order is NULL");
    return decode_common(H, llr, n, k, budget, batch, order, codeword, queries, abandoned, stream);
}

int orbg_schedule_export(int n, uint64_t count, uint8_t* out, void* stream)
{
    g_err.clear();
    if (n < 1 || n > ORBG_NMAX) return fail(ORBG_EINVAL, "n = %d outside [1, %d]", n, ORBG_NMAX);
    if (count < 1 || count > ORBG_BUDGET_MAX || (n < 63 && count > (1ull << n)))
        return fail(ORBG_EINVAL, "count = %llu out of range", (unsigned long long)count);
    if (!out) return fail(ORBG_EINVAL, "out is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const orbg::Schedule* s = nullptr;
    int rc = get_schedule(n, count, st, &s);
    if (rc) return rc;
    uint8_t* d_out = nullptr;
    if (hipMalloc(&d_out, 16 * count) != hipSuccess) return fail(ORBG_ENOMEM, "cannot allocate export buffer");
    const bool ok = orbg::orbg_unpack_schedule(s, count, d_out, st) == 0 &&
                    hipMemcpyAsync(out, d_out, 16 * count, hipMemcpyDeviceToHost, st) == hipSuccess &&
                    hipStreamSynchronize(st) == hipSuccess;
    (void)hipFree(d_out);
    if (!ok) return fail(ORBG_EHIP, "schedule export failed");
    return ORBG_OK;
}

const char* orbg_last_error(void) { return g_err.c_str(); }

}  // extern "C"
