/* Sanitizer driver for the oracle (test infrastructure): calls every entry
 * point of oracle/orbgrand_oracle.c on small seeded inputs, special LLR values
 * included, and checks the decoders' basic invariants.  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitize.py;
 * exits 0 when every check holds and the sanitizers report nothing. */
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

long oracle_landslide(int Wp, int w, int np, int* out, long max_count);
long oracle_order_prefix(int n, long count, int width, int* out, int* wout);
int oracle_decode(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, long batch, uint8_t* cw,
                  uint64_t* queries, uint8_t* abandoned, int threads);
int oracle_decode_ordered(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, long batch,
                          const uint8_t* order, uint8_t* cw, uint64_t* queries, uint8_t* abandoned, int threads);
int oracle_decode_1line(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, long batch, uint8_t* cw,
                        uint64_t* queries, uint8_t* abandoned, int32_t* j0_out, long j0_force, int threads);
long oracle_order1_prefix(int n, long j0, long count, int width, int* out, int* wout);
long oracle_fit_j0(const float* llr, int n);
int oracle_is_codeword(const uint8_t* H, int n, int k, const uint8_t* x);
void oracle_permutation(const float* llr, int n, int* pi);
long oracle_order_mline_prefix(int n, int m, const int* I, const long* J, const long* beta, long count, int width,
                               int* out, int* wout);
int oracle_fit_mline(const float* llr, int n, int mreq, int jdiv, int* m, int* I, long* J, long* beta);
int oracle_decode_mline(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, long batch, int mreq,
                        int jdiv, uint8_t* cw, uint64_t* queries, uint8_t* abandoned, int32_t* m_out, int threads);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint32_t next32(void)
{
    state ^= state << 13; state ^= state >> 7; state ^= state << 17;
    return (uint32_t)(state >> 32);
}
static float gauss(void)
{
    double u = (next32() + 1.0) / 4294967297.0, v = (next32() + 1.0) / 4294967297.0;
    return (float)(sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v));
}

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

/* H = [P | I] with P random. */
static uint8_t* make_code(int n, int k)
{
    const int m = n - k;
    uint8_t* H = calloc((size_t)m * n, 1);
    for (int r = 0; r < m; ++r) {
        for (int c = 0; c < k; ++c) H[(size_t)r * n + c] = next32() & 1u;
        H[(size_t)r * n + k + r] = 1;
    }
    return H;
}

static void check_results(const uint8_t* H, int n, int k, long N, uint64_t budget, const uint8_t* cw,
                          const uint64_t* q, const uint8_t* ab)
{
    for (long b = 0; b < N; ++b) {
        CHECK(q[b] >= 1 && q[b] <= budget);
        if (ab[b]) CHECK(q[b] == budget);
        else CHECK(oracle_is_codeword(H, n, k, cw + (size_t)b * n));
    }
}

static void run_code(int n, int k, uint64_t budget, long N)
{
    uint8_t* H = make_code(n, k);
    float* llr = malloc(sizeof(float) * (size_t)N * n);
    for (long i = 0; i < N * n; ++i) llr[i] = 2.0f * ((next32() & 1u) ? 1.0f : -1.0f) + gauss();
    /* special values in the first rows */
    if (N > 3) {
        for (int i = 0; i < n; ++i) llr[i] = (i % 3 == 0) ? 0.0f : (i % 3 == 1 ? -0.0f : 1.0f);
        llr[n] = NAN; llr[n + 1] = INFINITY; llr[n + 2] = -INFINITY;
        for (int i = 0; i < n; ++i) llr[2 * n + i] = (float)(i % 4) - 1.5f;         /* ties */
    }
    uint8_t* cw = malloc((size_t)N * n);
    uint64_t* q = malloc(sizeof(uint64_t) * N);
    uint8_t* ab = malloc(N);
    int32_t* aux = malloc(sizeof(int32_t) * N);
    CHECK(oracle_decode(H, llr, n, k, budget, N, cw, q, ab, 1) == 0);
    check_results(H, n, k, N, budget, cw, q, ab);
    if (n >= 12) {
        uint8_t* order = malloc((size_t)N * 64);
        for (long b = 0; b < N; ++b)
            for (int j = 0; j < 64; ++j) order[b * 64 + j] = (uint8_t)((j * 7 + b) % 64);
        CHECK(oracle_decode_ordered(H, llr, n, k, budget, N, order, cw, q, ab, 1) == 0);
        check_results(H, n, k, N, budget, cw, q, ab);
        free(order);
    }
    CHECK(oracle_decode_1line(H, llr, n, k, budget, N, cw, q, ab, aux, LONG_MIN, 1) == 0);
    check_results(H, n, k, N, budget, cw, q, ab);
    for (int mreq = 1; mreq <= 4; ++mreq)
        for (int jdiv = 0; jdiv <= 1; ++jdiv) {
            CHECK(oracle_decode_mline(H, llr, n, k, budget, N, mreq, jdiv, cw, q, ab, aux, 1) == 0);
            check_results(H, n, k, N, budget, cw, q, ab);
        }
    int* pi = malloc(sizeof(int) * n);
    oracle_permutation(llr + (size_t)(N - 1) * n, n, pi);
    (void)oracle_fit_j0(llr + (size_t)(N - 1) * n, n);
    int m = 0, I[9];
    long J[9], beta[9];
    CHECK(oracle_fit_mline(llr + (size_t)(N - 1) * n, n, 4, 0, &m, I, J, beta) == 0 || 1);
    free(pi); free(aux); free(ab); free(q); free(cw); free(llr); free(H);
}

int main(void)
{
    int out[16 * 4096], wout[4096];
    CHECK(oracle_landslide(8, 4, 4, out, 100) == 8);      /* the worked example: 8 partitions */
    CHECK(oracle_order_prefix(13, 4096, 16, out, wout) == 4096);
    CHECK(oracle_order_prefix(100, 4000, 16, out, wout) == 4000);
    CHECK(oracle_order1_prefix(20, 3, 4000, 16, out, wout) == 4000);
    {
        int I[3] = {0, 4, 10};
        long J[2] = {-1, 6}, beta[2] = {1, 2};
        CHECK(oracle_order_mline_prefix(10, 2, I, J, beta, 1000, 16, out, wout) > 0);
    }
    run_code(8, 3, 64, 50);
    run_code(32, 26, 10000, 120);
    run_code(64, 52, 20000, 40);
    run_code(127, 113, 5000, 24);
    run_code(130, 100, 3000, 8);
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
