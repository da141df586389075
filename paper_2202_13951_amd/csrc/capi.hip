// C-ABI front end of liborbgrand: argument checks, device caches of packed
// parity-check columns and query schedules, per-stream work space, kernel
// launches.
#include "orbgrand.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "orbg_internal.h"
#include "orbg_kernels.h"
#include "orbg_mlp.h"
#include "orbg_mline.h"

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
    int dev = 0;
    int n = 0, k = 0;
    std::vector<uint8_t> H;     // host copy, for exact cache matching
    uint64_t* d_cols = nullptr; // n columns: bit r of column i = H[r][i]
    uint64_t* d_rows = nullptr; // (n - k) x nk words: bit l of word j of row r = H[r][64 j + l]
};

int keys_per_lane(int n);

struct Workspace {
    unsigned long long* ctrs = nullptr;
    int64_t* heavy = nullptr;
    int64_t heavy_cap = 0;
};

std::mutex g_mu;
// (device, hash) -> codes with that hash
std::map<std::pair<int, uint64_t>, std::vector<CodeEntry*>> g_codes;
// registered code ids -> code
std::vector<CodeEntry*> g_registry;
// (device, n, len) -> schedule
std::map<std::tuple<int, int, uint64_t>, orbg::Schedule*> g_sched;
// (device, n, len) -> 1-line schedules
std::map<std::tuple<int, int, uint64_t>, orbg::Schedule1*> g_sched1;
// (device, n, length) whose 1-line order the per-offset schedules cannot hold
std::set<std::tuple<int, int, uint64_t>> g_sched1_no;
// (device, stream) -> work space
std::map<std::pair<int, hipStream_t>, Workspace> g_work;
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
int get_code(const uint8_t* H, int n, int k, CodeEntry** out)
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
        if (c->n == n && c->k == k && std::memcmp(c->H.data(), H, sz) == 0) { *out = c; return ORBG_OK; }
    std::vector<uint64_t> packed(n, 0ull);
    for (int r = 0; r < n - k; ++r)
        for (int i = 0; i < n; ++i)
            if (H[(size_t)r * n + i]) packed[i] |= 1ull << r;
    CodeEntry* c = new CodeEntry;
    c->dev = dev;
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
    const int nk = keys_per_lane(n);
    std::vector<uint64_t> rows((size_t)(n - k) * nk, 0ull);
    for (int r = 0; r < n - k; ++r)
        for (int i = 0; i < n; ++i)
            if (H[(size_t)r * n + i]) rows[(size_t)r * nk + i / 64] |= 1ull << (i % 64);
    if (hipMalloc(&c->d_rows, sizeof(uint64_t) * rows.size()) != hipSuccess) {
        (void)hipFree(c->d_cols);
        delete c;
        return fail(ORBG_ENOMEM, "cannot allocate %zu packed row words", rows.size());
    }
    if (hipMemcpy(c->d_rows, rows.data(), sizeof(uint64_t) * rows.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->d_cols);
        (void)hipFree(c->d_rows);
        delete c;
        return fail(ORBG_EHIP, "copy of packed rows failed");
    }
    bucket.push_back(c);
    *out = c;
    return ORBG_OK;
}

uint64_t round_up_pow2(uint64_t x)
{
    uint64_t p = 64;
    while (p < x) p <<= 1;
    return p;
}

// Schedule with at least `need` entries for length n (need <= 2^n).  build =
// false only looks it up (ORBG_EINVAL if it has not been built yet).
int get_schedule(int n, uint64_t need, hipStream_t stream, const orbg::Schedule** out, bool build = true)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ORBG_EHIP, "hipGetDevice failed");
    // lengths up to 2^22 are powers of two (budgets share schedules); longer
    // ones whole batches of 64
    uint64_t len = need <= ORBG_SCHED_POW2_MAX ? round_up_pow2(need) : (need + 63) / 64 * 64;
    if (n < 63 && len > (1ull << n)) len = 1ull << n;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(dev, n, len);
    auto it = g_sched.find(key);
    if (it != g_sched.end()) { *out = it->second; return ORBG_OK; }
    if (!build)
        return fail(ORBG_EINVAL, "no query schedule for n = %d and this budget on device %d yet (a call of "
                    "orbg_decode_mixed with the same codes and budget builds it)", n, dev);
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

// 1-line schedules with at least `need` entries for length n (need <= 2^n):
// lengths are whole batches of 64, so budgets within one batch share them.
int get_schedule_1line(int n, uint64_t need, hipStream_t stream, const orbg::Schedule1** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ORBG_EHIP, "hipGetDevice failed");
    uint64_t len = (need + 63) / 64 * 64;
    if (n < 63 && len > (1ull << n)) len = 1ull << n;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(dev, n, len);
    auto it = g_sched1.find(key);
    if (it != g_sched1.end()) { *out = it->second; return ORBG_OK; }
    if (g_sched1_no.count(key))
        return fail(ORBG_EINVAL, "1-line schedule: the order of %llu patterns at n = %d does not fit the schedules",
                    (unsigned long long)len, n);
    orbg::Schedule1* s = new orbg::Schedule1;
    char err[256] = {0};
    const int rc = orbg_build_schedule_1line(n, len, stream, s, err, sizeof(err));
    if (rc != 0) {
        delete s;
        if (rc == -1) g_sched1_no.insert(key);
        return fail(rc == -2 ? ORBG_ENOMEM : (rc == -1 ? ORBG_EINVAL : ORBG_EHIP), "%s", err);
    }
    g_sched1[key] = s;
    *out = s;
    return ORBG_OK;
}

// Per-stream counters and heavy-block list (calls on one stream are ordered,
// so they can share them).  Grows the list to `heavy_need` entries.
int get_workspace(hipStream_t st, int64_t heavy_need, Workspace** out, int* cus)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ORBG_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace& w = g_work[{dev, st}];
    if (!w.ctrs && hipMalloc(&w.ctrs, sizeof(unsigned long long) * ORBG_CTR_WORDS) != hipSuccess) {
        w.ctrs = nullptr;
        return fail(ORBG_ENOMEM, "cannot allocate work counters");
    }
    if (heavy_need > w.heavy_cap) {
        // the old list may still be read by work queued on this stream
        if (w.heavy && (hipStreamSynchronize(st) != hipSuccess || hipFree(w.heavy) != hipSuccess))
            return fail(ORBG_EHIP, "cannot release the heavy-block list");
        w.heavy = nullptr;
        w.heavy_cap = 0;
        if (hipMalloc(&w.heavy, sizeof(int64_t) * heavy_need) != hipSuccess) {
            w.heavy = nullptr;
            return fail(ORBG_ENOMEM, "cannot allocate a heavy-block list of %lld entries", (long long)heavy_need);
        }
        w.heavy_cap = heavy_need;
    }
    *out = &w;
    auto c = g_cus.find(dev);
    if (c == g_cus.end()) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1) v = 256;
        c = g_cus.emplace(dev, v).first;
    }
    *cus = c->second;
    return ORBG_OK;
}

orbg::LaunchParams resolve_params(const orbg_launch_params* p, bool ordered)
{
    orbg::LaunchParams r;
    r.wg_per_cu = 32;
    r.chunk = 0;
    r.split_steps = 64;
    r.heavy_waves = 8;
    r.heavy_wg_per_cu = 2;
    r.naive = 0;
    if (p) {
        if (p->workgroups_per_cu > 0) r.wg_per_cu = p->workgroups_per_cu;
        if (p->chunk > 0) r.chunk = p->chunk;
        if (p->split_steps >= 0) r.split_steps = p->split_steps;
        if (p->heavy_waves > 0) r.heavy_waves = p->heavy_waves;
        if (p->heavy_workgroups_per_cu > 0) r.heavy_wg_per_cu = p->heavy_workgroups_per_cu;
        r.naive = p->one_block_per_workgroup;
        if (r.naive) r.split_steps = 0;
    }
    // the reordered prefix (64 steps) always stays in the light pass
    if (ordered && r.split_steps > 0 && r.split_steps < 64) r.split_steps = 64;
    return r;
}

int check_params(const orbg_launch_params* p)
{
    if (!p) return ORBG_OK;
    if (p->workgroups_per_cu < 0 || p->workgroups_per_cu > 64)
        return fail(ORBG_EINVAL, "workgroups_per_cu = %d outside [0, 64]", p->workgroups_per_cu);
    if (p->chunk < 0 || p->chunk > 64) return fail(ORBG_EINVAL, "chunk = %d outside [0, 64]", p->chunk);
    if (p->split_steps < -1) return fail(ORBG_EINVAL, "split_steps = %d below -1", p->split_steps);
    if (p->heavy_waves != 0 && p->heavy_waves != 4 && p->heavy_waves != 8 && p->heavy_waves != 16)
        return fail(ORBG_EINVAL, "heavy_waves = %d is not 0, 4, 8 or 16", p->heavy_waves);
    if (p->heavy_workgroups_per_cu < 0 || p->heavy_workgroups_per_cu > 16)
        return fail(ORBG_EINVAL, "heavy_workgroups_per_cu = %d outside [0, 16]", p->heavy_workgroups_per_cu);
    if (p->one_block_per_workgroup != 0 && p->one_block_per_workgroup != 1)
        return fail(ORBG_EINVAL, "one_block_per_workgroup = %d is not 0 or 1", p->one_block_per_workgroup);
    return ORBG_OK;
}

int keys_per_lane(int n)
{
    int nk = 1;
    while (nk * 64 < n) nk <<= 1;
    return nk;
}

// Fills one code descriptor (schedule for `need` queries; build = false: the
// schedule must exist already).
int describe(const CodeEntry* c, uint64_t need, hipStream_t st, uint32_t col_base, orbg::CodeDesc* d,
             bool build = true)
{
    if (c->n < 63 && need > (1ull << c->n)) need = 1ull << c->n;
    const orbg::Schedule* s = nullptr;
    int rc = get_schedule(c->n, need, st, &s, build);
    if (rc) return rc;
    d->n = c->n;
    d->m = c->n - c->k;
    d->nk = keys_per_lane(c->n);
    d->rdepth = s->rmax < c->n ? s->rmax : c->n;
    d->rdepth0 = s->rmax0 < d->rdepth ? s->rmax0 : d->rdepth;
    d->slen = (uint32_t)s->len;
    d->col_base = col_base;
    d->cols = c->d_cols;
    d->rows = c->d_rows;
    d->row_base = 0;
    d->sched = s->entries;
    return ORBG_OK;
}

// Code descriptor of a 1-line decode (schedules for `need` queries).
int describe_1line(const CodeEntry* c, uint64_t need, hipStream_t st, orbg::CodeDesc* d)
{
    if (c->n < 63 && need > (1ull << c->n)) need = 1ull << c->n;
    const orbg::Schedule1* s = nullptr;
    int rc = get_schedule_1line(c->n, need, st, &s);
    if (rc) return rc;
    d->n = c->n;
    d->m = c->n - c->k;
    d->nk = keys_per_lane(c->n);
    d->rdepth = s->rmax < c->n ? s->rmax : c->n;
    d->rdepth0 = d->rdepth;
    d->slen = (uint32_t)s->len;
    d->col_base = 0;
    d->cols = c->d_cols;
    d->rows = c->d_rows;
    d->row_base = 0;
    d->sched = s->entries;
    d->j0max = s->j0max;
    d->sstride = (uint32_t)s->stride;
    return ORBG_OK;
}

int check_budget(uint64_t budget, int64_t batch)
{
    if (budget < 1 || budget > ORBG_BUDGET_MAX)
        return fail(ORBG_EINVAL, "budget = %llu outside [1, 5 x 10^6]", (unsigned long long)budget);
    if (batch < 0) return fail(ORBG_EINVAL, "batch = %lld is negative", (long long)batch);
    return ORBG_OK;
}

// device -> subset-count table of the m-line order (built once per device)
std::map<int, uint32_t*> g_ml_table;

int get_ml_table(hipStream_t st, const uint32_t** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ORBG_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ml_table.find(dev);
    if (it != g_ml_table.end()) { *out = it->second; return ORBG_OK; }
    uint32_t* t = nullptr;
    if (hipMalloc(&t, sizeof(uint32_t) * orbg::subset_table_words()) != hipSuccess)
        return fail(ORBG_ENOMEM, "cannot allocate the subset-count table");
    hipError_t e = orbg::build_subset_table(t, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(t);
        return fail(ORBG_EHIP, "subset-count table build failed: %s", hipGetErrorString(e));
    }
    g_ml_table.emplace(dev, t);
    *out = t;
    return ORBG_OK;
}

// Scratch of the allocation-free mixed decode: the work counters (ORBG_CTR_WORDS
// words), then the heavy-block list (one i64 per block).  Each device holds its
// own copy for the life of the process; calls on one device share it.
static_assert(ORBG_NOALLOC_BATCH_MAX == (1 << 18), "scratch size");
static __device__ __align__(256) unsigned long long scratch[ORBG_CTR_WORDS + ORBG_NOALLOC_BATCH_MAX];

// device -> device address of `scratch` on it (the host-side name is only a
// stand-in for the symbol: kernels get this address)
std::map<int, unsigned long long*> g_scratch;

int get_scratch(int dev, unsigned long long** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) { *out = it->second; return ORBG_OK; }
    unsigned long long* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        return fail(ORBG_EHIP, "cannot find the scratch array on device %d: %s", dev, hipGetErrorString(e));
    g_scratch.emplace(dev, ptr);
    *out = ptr;
    return ORBG_OK;
}

int compute_units(int dev, int* cus)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto c = g_cus.find(dev);
    if (c == g_cus.end()) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1) v = 256;
        c = g_cus.emplace(dev, v).first;
    }
    *cus = c->second;
    return ORBG_OK;
}

// Full m-line decode of a checked request (n <= ORBG_ML_LMAX, budget <=
// ORBG_ML_BUDGET_MAX, segments and jdiv in range).  j0: per-block J_0 of the
// fit, or NULL.
int decode_mline_checked(const CodeEntry* code, const float* llr, uint64_t budget, int64_t batch, int segments,
                         int jdiv, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned, int32_t* segments_out,
                         int32_t* j0, hipStream_t st)
{
    int rc;
    const uint32_t* tbl = nullptr;
    if ((rc = get_ml_table(st, &tbl))) return rc;
    if (batch == 0) return ORBG_OK;
    Workspace* w = nullptr;
    int cus = 0;
    if ((rc = get_workspace(st, 0, &w, &cus))) return rc;
    orbg::MlineArgs a;
    a.llr = llr;
    a.n = code->n;
    a.m = code->n - code->k;
    a.cols = code->d_cols;
    a.rows = code->d_rows;
    a.nblocks = batch;
    a.budget = (uint32_t)budget;
    a.mseg = segments;
    a.jdiv = jdiv != 0;
    a.table = tbl;
    a.cw = codeword;
    a.queries = queries;
    a.abandoned = abandoned;
    a.mfit = segments_out;
    a.j0 = j0;
    // one-wave workgroups, several times more than fit at once: each takes a
    // strided share of the blocks, and the hardware hands out the later
    // workgroups as earlier ones finish, which evens out blocks of unequal cost
    // (measured: 96 per CU decodes the 4 dB BCH point 1.2x faster than 32)
    const int64_t grid = std::min<int64_t>(batch, (int64_t)cus * 96);
    const hipError_t e = orbg::launch_mline(a, (int)grid, st);
    if (e != hipSuccess) return fail(ORBG_EHIP, "m-line decode launch failed: %s", hipGetErrorString(e));
    return ORBG_OK;
}

int decode_single(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                  const uint8_t* order, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned,
                  const orbg_launch_params* params, void* stream, bool oneline = false, int32_t* j0 = nullptr)
{
    int rc = check_code_args(H, n, k);
    if (rc) return rc;
    if ((rc = check_budget(budget, batch)) || (rc = check_params(params))) return rc;
    if (batch > 0 && (!llr || !codeword || !queries || !abandoned))
        return fail(ORBG_EINVAL, "a device buffer is NULL");
    if (order && n < 12) return fail(ORBG_EINVAL, "a batch order needs n >= 12 (got %d)", n);
    if (oneline && budget > ORBG_BUDGET_MAX_1LINE && n > ORBG_ML_LMAX)
        return fail(ORBG_EINVAL, "budget = %llu above 2^22, the 1-line schedules' limit, and n = %d above %d for "
                    "the one-segment m-line decode", (unsigned long long)budget, n, ORBG_ML_LMAX);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CodeEntry* code = nullptr;
    if ((rc = get_code(H, n, k, &code))) return rc;
    orbg::DecodeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.codes.ncodes = 1;
    if (oneline) {
        // 1-line ORBGRAND is full ORBGRAND with one segment (the same fit and
        // order): where the per-offset schedules cannot hold the order of
        // (n, budget), the m-line kernel decodes with one segment
        rc = budget <= ORBG_BUDGET_MAX_1LINE ? describe_1line(code, budget, st, &a.codes.c[0]) : ORBG_EINVAL;
        if (rc == ORBG_EINVAL && n <= ORBG_ML_LMAX) {
            g_err.clear();
            return decode_mline_checked(code, llr, budget, batch, 1, 0, codeword, queries, abandoned, nullptr, j0,
                                        st);
        }
    } else {
        rc = describe(code, order && budget < 4096 ? 4096 : budget, st, 0, &a.codes.c[0]);
    }
    if (rc) return rc;
    a.codes.rwords = a.codes.c[0].m * a.codes.c[0].nk;
    if (batch == 0) return ORBG_OK;
    a.p = resolve_params(params, order != nullptr);
    Workspace* w = nullptr;
    if ((rc = get_workspace(st, a.p.split_steps > 0 ? batch : 0, &w, &a.cus))) return rc;
    a.mixed = false;
    a.llr = llr;
    a.nblocks = batch;
    a.budget = (uint32_t)budget;
    a.order = order;
    a.oneline = oneline;
    a.j0 = j0;
    a.cw = codeword;
    a.queries = queries;
    a.abandoned = abandoned;
    a.ctrs = w->ctrs;
    a.heavy = a.p.split_steps > 0 ? w->heavy : nullptr;
    const hipError_t e = orbg::launch_decode(a, st);
    if (e != hipSuccess) return fail(ORBG_EHIP, "decode launch failed: %s", hipGetErrorString(e));
    return ORBG_OK;
}

// Mixed-code decode.  noalloc: no device allocation of any kind -- the
// schedules must exist already, and the work counters and heavy-block list
// live in this device's `scratch` array (batch <= ORBG_NOALLOC_BATCH_MAX).
int decode_mixed(const int* codes, int ncodes, const uint8_t* block_code, const int64_t* row_offset,
                 const float* llr, int64_t llr_len, int64_t batch, uint64_t budget, uint8_t* codeword,
                 int64_t codeword_len, uint64_t* queries, uint8_t* abandoned, const orbg_launch_params* params,
                 void* stream, bool noalloc)
{
    int rc = check_budget(budget, batch);
    if (rc || (rc = check_params(params))) return rc;
    if (llr_len < 0 || codeword_len < 0)
        return fail(ORBG_EINVAL, "buffer lengths %lld (llr) and %lld (codeword) must not be negative",
                    (long long)llr_len, (long long)codeword_len);
    if (noalloc && batch > ORBG_NOALLOC_BATCH_MAX)
        return fail(ORBG_EINVAL, "batch = %lld above %d, the most the allocation-free decode takes",
                    (long long)batch, ORBG_NOALLOC_BATCH_MAX);
    if (!codes || ncodes < 1 || ncodes > ORBG_MAX_CODES)
        return fail(ORBG_EINVAL, "ncodes = %d outside [1, %d]", ncodes, ORBG_MAX_CODES);
    if (batch > 0 && (!block_code || !row_offset || !llr || !codeword || !queries || !abandoned))
        return fail(ORBG_EINVAL, "a device buffer is NULL");
    CodeEntry* list[ORBG_MAX_CODES];
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (int i = 0; i < ncodes; ++i) {
            if (codes[i] < 0 || codes[i] >= (int)g_registry.size() || !g_registry[codes[i]])
                return fail(ORBG_EINVAL, "code id %d is not registered", codes[i]);
            list[i] = g_registry[codes[i]];
            if (list[i]->n > 256) return fail(ORBG_EINVAL, "mixed decodes take n <= 256 (code %d)", codes[i]);
        }
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ORBG_EHIP, "hipGetDevice failed");
    for (int i = 0; i < ncodes; ++i)
        if (list[i]->dev != dev) return fail(ORBG_EINVAL, "code id %d lives on another device", codes[i]);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    orbg::DecodeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.codes.ncodes = ncodes;
    uint32_t col_base = 0, row_base = 0;
    for (int i = 0; i < ncodes; ++i) {
        if ((rc = describe(list[i], budget, st, col_base, &a.codes.c[i], !noalloc))) return rc;
        a.codes.c[i].row_base = row_base;
        col_base += (uint32_t)list[i]->n;
        row_base += (uint32_t)(a.codes.c[i].m * a.codes.c[i].nk);
    }
    a.codes.rwords = (int)row_base;
    if (col_base > ORBG_MIXED_COLS)
        return fail(ORBG_EINVAL, "the codes of one mixed decode may hold at most %d columns", ORBG_MIXED_COLS);
    unsigned long long* scr = nullptr;
    if (noalloc && (rc = get_scratch(dev, &scr))) return rc;
    if (batch == 0) return ORBG_OK;
    a.p = resolve_params(params, false);
    if (noalloc) {
        if ((rc = compute_units(dev, &a.cus))) return rc;
        a.ctrs = scr;
        a.heavy = a.p.split_steps > 0 ? reinterpret_cast<int64_t*>(scr + ORBG_CTR_WORDS) : nullptr;
    } else {
        Workspace* w = nullptr;
        if ((rc = get_workspace(st, a.p.split_steps > 0 ? batch : 0, &w, &a.cus))) return rc;
        a.ctrs = w->ctrs;
        a.heavy = a.p.split_steps > 0 ? w->heavy : nullptr;
    }
    a.mixed = true;
    a.block_code = block_code;
    a.row_off = row_offset;
    a.row_limit = llr_len < codeword_len ? llr_len : codeword_len;
    a.llr = llr;
    a.nblocks = batch;
    a.budget = (uint32_t)budget;
    a.order = nullptr;
    a.cw = codeword;
    a.queries = queries;
    a.abandoned = abandoned;
    const hipError_t e = orbg::launch_decode(a, st);
    if (e != hipSuccess) return fail(ORBG_EHIP, "mixed decode launch failed: %s", hipGetErrorString(e));
    return ORBG_OK;
}

}  // namespace

extern "C" {

int orbg_decode(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                uint8_t* codeword, uint64_t* queries, uint8_t* abandoned, void* stream)
{
    g_err.clear();
    return decode_single(H, llr, n, k, budget, batch, nullptr, codeword, queries, abandoned, nullptr, stream);
}

int orbg_decode_ordered(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                        const uint8_t* order, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned,
                        void* stream)
{
    g_err.clear();
    if (!order && batch > 0) return fail(ORBG_EINVAL, "order is NULL");
    return decode_single(H, llr, n, k, budget, batch, order, codeword, queries, abandoned, nullptr, stream);
}

int orbg_decode_ex(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                   const uint8_t* order, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned,
                   const orbg_launch_params* params, void* stream)
{
    g_err.clear();
    return decode_single(H, llr, n, k, budget, batch, order, codeword, queries, abandoned, params, stream);
}

int orbg_decode_1line(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                      uint8_t* codeword, uint64_t* queries, uint8_t* abandoned, int32_t* j0,
                      const orbg_launch_params* params, void* stream)
{
    g_err.clear();
    return decode_single(H, llr, n, k, budget, batch, nullptr, codeword, queries, abandoned, params, stream, true,
                         j0);
}

int orbg_decode_mline(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                      int segments, int jdiv, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned,
                      int32_t* segments_out, void* stream)
{
    g_err.clear();
    int rc = check_code_args(H, n, k);
    if (rc) return rc;
    if (n > ORBG_ML_LMAX) return fail(ORBG_EINVAL, "n = %d above %d for the m-line order", n, ORBG_ML_LMAX);
    if (segments < 1 || segments > ORBG_ML_MSEG)
        return fail(ORBG_EINVAL, "segments = %d outside [1, %d]", segments, ORBG_ML_MSEG);
    if (jdiv != 0 && jdiv != 1) return fail(ORBG_EINVAL, "jdiv = %d is not 0 or 1", jdiv);
    if (budget < 1 || budget > ORBG_ML_BUDGET_MAX)
        return fail(ORBG_EINVAL, "budget = %llu outside [1, 5 x 10^6] for the m-line order", (unsigned long long)budget);
    if (batch < 0) return fail(ORBG_EINVAL, "batch = %lld is negative", (long long)batch);
    if (batch > 0 && (!llr || !codeword || !queries || !abandoned))
        return fail(ORBG_EINVAL, "a device buffer is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CodeEntry* code = nullptr;
    if ((rc = get_code(H, n, k, &code))) return rc;
    return decode_mline_checked(code, llr, budget, batch, segments, jdiv, codeword, queries, abandoned, segments_out,
                                nullptr, st);
}

int orbg_code_register(const uint8_t* H, int n, int k, int* code_id)
{
    g_err.clear();
    int rc = check_code_args(H, n, k);
    if (rc) return rc;
    if (!code_id) return fail(ORBG_EINVAL, "code_id is NULL");
    CodeEntry* c = nullptr;
    if ((rc = get_code(H, n, k, &c))) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = 0; i < g_registry.size(); ++i)
        if (!g_registry[i]) { g_registry[i] = c; *code_id = (int)i; return ORBG_OK; }
    g_registry.push_back(c);
    *code_id = (int)g_registry.size() - 1;
    return ORBG_OK;
}

int orbg_code_release(int code_id)
{
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_mu);
    if (code_id < 0 || code_id >= (int)g_registry.size() || !g_registry[code_id])
        return fail(ORBG_EINVAL, "code id %d is not registered", code_id);
    g_registry[code_id] = nullptr;     // the packed columns stay cached by content
    return ORBG_OK;
}

int orbg_decode_mixed(const int* codes, int ncodes, const uint8_t* block_code, const int64_t* row_offset,
                      const float* llr, int64_t llr_len, int64_t batch, uint64_t budget, uint8_t* codeword,
                      int64_t codeword_len, uint64_t* queries, uint8_t* abandoned, const orbg_launch_params* params,
                      void* stream)
{
    g_err.clear();
    return decode_mixed(codes, ncodes, block_code, row_offset, llr, llr_len, batch, budget, codeword, codeword_len,
                        queries, abandoned, params, stream, false);
}

int orbg_decode_mixed_noalloc(const int* codes, int ncodes, const uint8_t* block_code, const int64_t* row_offset,
                              const float* llr, int64_t llr_len, int64_t batch, uint64_t budget, uint8_t* codeword,
                              int64_t codeword_len, uint64_t* queries, uint8_t* abandoned,
                              const orbg_launch_params* params, void* stream)
{
    g_err.clear();
    return decode_mixed(codes, ncodes, block_code, row_offset, llr, llr_len, batch, budget, codeword, codeword_len,
                        queries, abandoned, params, stream, true);
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

int orbg_schedule_export_1line(int n, uint64_t budget, int j0, uint64_t count, uint8_t* out, int* j0max,
                               void* stream)
{
    g_err.clear();
    if (n < 1 || n > ORBG_NMAX) return fail(ORBG_EINVAL, "n = %d outside [1, %d]", n, ORBG_NMAX);
    if (budget < 1 || budget > ORBG_BUDGET_MAX_1LINE || (n < 63 && budget > (1ull << n)))
        return fail(ORBG_EINVAL, "budget = %llu out of range", (unsigned long long)budget);
    if (count > budget) return fail(ORBG_EINVAL, "count = %llu above the budget", (unsigned long long)count);
    if (j0 < -1 || j0 >= (1 << 20)) return fail(ORBG_EINVAL, "j0 = %d outside [-1, 2^20 - 1]", j0);
    if (count > 0 && !out) return fail(ORBG_EINVAL, "out is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const orbg::Schedule1* s = nullptr;
    int rc = get_schedule_1line(n, budget, st, &s);
    if (rc) return rc;
    if (j0max) *j0max = s->j0max;
    if (count == 0) return ORBG_OK;
    const int jc = j0 < s->j0max ? j0 : s->j0max;
    uint8_t* d_out = nullptr;
    if (hipMalloc(&d_out, 16 * count) != hipSuccess) return fail(ORBG_ENOMEM, "cannot allocate export buffer");
    const bool ok = orbg::orbg_unpack_entries(s->entries + (size_t)(jc + 1) * s->stride, count, d_out, st) == 0 &&
                    hipMemcpyAsync(out, d_out, 16 * count, hipMemcpyDeviceToHost, st) == hipSuccess &&
                    hipStreamSynchronize(st) == hipSuccess;
    (void)hipFree(d_out);
    if (!ok) return fail(ORBG_EHIP, "schedule export failed");
    return ORBG_OK;
}

// Work space of a gated learned decode: the list of blocks left after batch 0,
// their feature rows and network activations (at most MLP_BATCH_MAX at a time)
// and their batch orders.
struct LearnedWs {
    int64_t* list;
    uint8_t* orders;
    int64_t bytes;
};

static LearnedWs learned_carve(void* base, int64_t batch)
{
    LearnedWs w;
    unsigned char* p = reinterpret_cast<unsigned char*>(base);
    int64_t o = 0;
    auto take = [&](int64_t bytes) { void* r = p ? p + o : nullptr; o += (bytes + 255) & ~(int64_t)255; return r; };
    w.list = (int64_t*)take(batch * 8);
    w.orders = (uint8_t*)take(batch * MLP_OUT);
    w.bytes = o;
    return w;
}

int64_t orbg_learned_workspace_bytes(int64_t batch)
{
    if (batch < 0) return -1;
    return learned_carve(nullptr, batch).bytes;
}

int orbg_decode_learned(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                        const float* w, const uint16_t* wb, void* workspace, int64_t workspace_bytes,
                        uint8_t* codeword, uint64_t* queries, uint8_t* abandoned, uint8_t* order_out, int64_t* rest,
                        const orbg_launch_params* params, void* stream)
{
    g_err.clear();
    int rc = check_code_args(H, n, k);
    if (rc || (rc = check_budget(budget, batch)) || (rc = check_params(params))) return rc;
    if (n != MLP_IN) return fail(ORBG_EINVAL, "the network takes n = %d (got %d)", MLP_IN, n);
    if (rest) *rest = 0;
    if (batch == 0) return ORBG_OK;
    if (!llr || !codeword || !queries || !abandoned || !w || !wb || !workspace)
        return fail(ORBG_EINVAL, "a device buffer is NULL");
    const LearnedWs need = learned_carve(nullptr, batch);
    if (workspace_bytes < need.bytes)
        return fail(ORBG_EINVAL, "work space of %lld bytes is smaller than the %lld needed", (long long)workspace_bytes,
                    (long long)need.bytes);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CodeEntry* code = nullptr;
    if ((rc = get_code(H, n, k, &code))) return rc;
    orbg::DecodeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.codes.ncodes = 1;
    if ((rc = describe(code, budget < 4096 ? 4096 : budget, st, 0, &a.codes.c[0]))) return rc;
    a.codes.rwords = a.codes.c[0].m * a.codes.c[0].nk;
    Workspace* ws = nullptr;
    if ((rc = get_workspace(st, 0, &ws, &a.cus))) return rc;
    const LearnedWs lw = learned_carve(workspace, batch);
    // 1. the first batch of the plain order for every block; the rest are listed
    a.p = resolve_params(params, false);
    a.p.split_steps = 1;
    a.llr = llr;
    a.nblocks = batch;
    a.budget = (uint32_t)budget;
    a.cw = codeword;
    a.queries = queries;
    a.abandoned = abandoned;
    a.ctrs = ws->ctrs;
    a.heavy = lw.list;
    a.list_only = true;
    hipError_t e = orbg::launch_decode(a, st);
    if (e != hipSuccess) return fail(ORBG_EHIP, "first-batch pass failed: %s", hipGetErrorString(e));
    unsigned long long count = 0;
    e = hipMemcpyAsync(&count, ws->ctrs + ORBG_CTR_HEAVY_COUNT, sizeof(count), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ORBG_EHIP, "reading the count of listed blocks failed: %s", hipGetErrorString(e));
    if (rest) *rest = (int64_t)count;
    // 2. features, network and batch order (batch 0 first) of the listed blocks,
    // one fused launch
    e = orbg::mlp_infer(w, wb, llr, batch, lw.list, nullptr, (int64_t)count, nullptr, lw.orders, true, st);
    if (e != hipSuccess) return fail(ORBG_EHIP, "network launch failed: %s", hipGetErrorString(e));
    if (order_out && (e = orbg::mlp_order_table(lw.orders, lw.list, (int64_t)count, batch, order_out, st)) != hipSuccess)
        return fail(ORBG_EHIP, "order table launch failed: %s", hipGetErrorString(e));
    if (count == 0) return ORBG_OK;
    // 3. ordered decode of the listed blocks from step 1 (blocks still open after
    // the split point, at least the 64 reordered batches, go to the heavy pass,
    // which indexes the caller's arrays directly)
    orbg::DecodeArgs b = a;
    b.p = resolve_params(params, true);
    if (b.p.split_steps > 0 && (rc = get_workspace(st, (int64_t)count, &ws, &b.cus))) return rc;
    b.ctrs = ws->ctrs;
    b.heavy = b.p.split_steps > 0 ? ws->heavy : nullptr;
    b.list_only = false;
    b.ids = lw.list;
    b.nblocks = (int64_t)count;
    b.order = lw.orders;
    b.skip0 = true;
    e = orbg::launch_decode(b, st);
    if (e != hipSuccess) return fail(ORBG_EHIP, "ordered pass failed: %s", hipGetErrorString(e));
    return ORBG_OK;
}

int64_t orbg_mlp_workspace_bytes(int64_t batch)
{
    if (batch < 0 || batch > MLP_BATCH_MAX) return -1;
    return orbg::mlp_carve(nullptr, batch).bytes;
}

int orbg_mlp_features(const float* llr, int n, int64_t batch, uint16_t* x, void* stream)
{
    g_err.clear();
    if (n != MLP_IN) return fail(ORBG_EINVAL, "features take n = %d (got %d)", MLP_IN, n);
    if (batch < 0) return fail(ORBG_EINVAL, "batch = %lld is negative", (long long)batch);
    if (batch > 0 && (!llr || !x)) return fail(ORBG_EINVAL, "a device buffer is NULL");
    const hipError_t e = orbg::mlp_features(llr, batch, x, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? ORBG_OK : fail(ORBG_EHIP, "features launch failed: %s", hipGetErrorString(e));
}

int orbg_mlp_prepare(const float* w, uint16_t* wb, uint16_t* wt, void* stream)
{
    g_err.clear();
    if (!w || !wb || !wt) return fail(ORBG_EINVAL, "a device buffer is NULL");
    const hipError_t e = orbg::mlp_prepare(w, wb, wt, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? ORBG_OK : fail(ORBG_EHIP, "prepare launch failed: %s", hipGetErrorString(e));
}

static int mlp_check(int64_t batch, void* workspace, int64_t workspace_bytes)
{
    if (batch < 0 || batch > MLP_BATCH_MAX)
        return fail(ORBG_EINVAL, "batch = %lld outside [0, %d]", (long long)batch, MLP_BATCH_MAX);
    if (batch > 0 && (!workspace || workspace_bytes < orbg::mlp_carve(nullptr, batch).bytes))
        return fail(ORBG_EINVAL, "work space of %lld bytes is smaller than the %lld needed", (long long)workspace_bytes,
                    (long long)orbg::mlp_carve(nullptr, batch).bytes);
    return ORBG_OK;
}

int orbg_mlp_forward(const float* w, const uint16_t* wb, const uint16_t* x, int64_t batch, float* logits,
                     void* workspace, int64_t workspace_bytes, void* stream)
{
    g_err.clear();
    int rc = mlp_check(batch, workspace, workspace_bytes);
    if (rc) return rc;
    if (batch > 0 && (!w || !wb || !x || !logits)) return fail(ORBG_EINVAL, "a device buffer is NULL");
    const hipError_t e = orbg::mlp_forward(w, wb, x, batch, logits, orbg::mlp_carve(workspace, batch),
                                           reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? ORBG_OK : fail(ORBG_EHIP, "forward launch failed: %s", hipGetErrorString(e));
}

int orbg_mlp_backward(const float* w, const uint16_t* wb, const uint16_t* wt, const uint16_t* x,
                      const int32_t* labels, int64_t batch, float* grads, float* loss, void* workspace,
                      int64_t workspace_bytes, void* stream)
{
    g_err.clear();
    int rc = mlp_check(batch, workspace, workspace_bytes);
    if (rc) return rc;
    if (batch < 1) return fail(ORBG_EINVAL, "the backward needs batch >= 1");
    if (!w || !wb || !wt || !x || !labels || !grads || !loss) return fail(ORBG_EINVAL, "a device buffer is NULL");
    const hipError_t e = orbg::mlp_backward(w, wb, wt, x, labels, batch, grads, loss,
                                            orbg::mlp_carve(workspace, batch), reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? ORBG_OK : fail(ORBG_EHIP, "backward launch failed: %s", hipGetErrorString(e));
}

int orbg_mlp_adam(float* w, float* m, float* v, const float* grads, float lr, int step, uint16_t* wb, uint16_t* wt,
                  void* stream)
{
    g_err.clear();
    if (!w || !m || !v || !grads || !wb || !wt) return fail(ORBG_EINVAL, "a device buffer is NULL");
    if (!(lr > 0.f) || lr > 1.f) return fail(ORBG_EINVAL, "lr = %g outside (0, 1]", (double)lr);
    if (step < 1) return fail(ORBG_EINVAL, "step = %d (steps count from 1)", step);
    const hipError_t e = orbg::mlp_adam(w, m, v, grads, lr, step, wb, wt, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? ORBG_OK : fail(ORBG_EHIP, "adam launch failed: %s", hipGetErrorString(e));
}

int orbg_mlp_infer(const float* w, const uint16_t* wb, const float* llr, int64_t llr_rows, const int64_t* ids,
                   const uint16_t* x, int64_t batch, float* logits, uint8_t* order, int pin0, void* stream)
{
    g_err.clear();
    if (batch < 0 || batch >= ((int64_t)1 << 31) * 32)
        return fail(ORBG_EINVAL, "batch = %lld outside [0, 2^36)", (long long)batch);
    if (llr && llr_rows < 0) return fail(ORBG_EINVAL, "llr_rows = %lld is negative", (long long)llr_rows);
    if (pin0 != 0 && pin0 != 1) return fail(ORBG_EINVAL, "pin0 = %d is not 0 or 1", pin0);
    if (!logits && !order) return fail(ORBG_EINVAL, "no output (logits and order are NULL)");
    if (batch == 0) return ORBG_OK;
    if (!w || !wb || (!llr && !x)) return fail(ORBG_EINVAL, "a device buffer is NULL");
    const hipError_t e = orbg::mlp_infer(w, wb, llr, llr_rows, llr ? ids : nullptr, llr ? nullptr : x, batch, logits,
                                         order, pin0 != 0, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? ORBG_OK : fail(ORBG_EHIP, "inference launch failed: %s", hipGetErrorString(e));
}

int orbg_mlp_order(const float* logits, int64_t batch, uint8_t* order, void* stream)
{
    g_err.clear();
    if (batch < 0) return fail(ORBG_EINVAL, "batch = %lld is negative", (long long)batch);
    if (batch > 0 && (!logits || !order)) return fail(ORBG_EINVAL, "a device buffer is NULL");
    const hipError_t e = orbg::mlp_order(logits, batch, order, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? ORBG_OK : fail(ORBG_EHIP, "order launch failed: %s", hipGetErrorString(e));
}

const char* orbg_last_error(void) { return g_err.c_str(); }

}  // extern "C"
