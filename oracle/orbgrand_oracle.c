/*
 * ORBGRAND CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately literal implementation of basic Ordered
 * Reliability Bits GRAND (Duffy, An, Medard, arXiv 2202.13951).  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this file's library.  The GPU decoder shares no code with it.
 *
 * What it follows, step by step:
 *   - GRAND driver: Algorithm 1 (query putative noise from most to least
 *     likely, stop at the first code-book member).
 *   - Hard decision and reliability: Sec. III-A (mod(c)=2c-1, LLR defined as
 *     log f(Y|1)/f(Y|0), y=(sign(LLR)+1)/2, reliability |LLR|), and the
 *     permutation pi of Sec. III-A (pi_i = received index of the i-th least
 *     reliable bit).
 *   - Query order: Sec. III-B, eqs. (lw) logistic weight, (znwl) weight
 *     classes S_W, (fractionation) split by Hamming weight, (intpart)/(vu)/
 *     (intpart2) shift to non-decreasing parts u with v_i = i + u_i.
 *   - Pattern generator: Sec. III-C, the Build-mountain routine (five steps)
 *     and the Landslide algorithm (Algorithm 2), run per (W, w).
 *   - Code-book membership for a linear code: Sec. I ("matrix multiplication
 *     and comparison"): H x = 0 over GF(2), computed row by row.
 *   - Abandonment: Sec. IV-A (a block is abandoned when no code-book member is
 *     found within the query budget).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   R1  LLR == 0 (either sign) and NaN give hard decision 0 (only LLR > 0 is 1).
 *   R2  Reliability ties are broken by the lower received index (stable sort).
 *       The sort key is (IEEE bits of |LLR|, index) compared lexicographically.
 *   R3  Inside one logistic weight W, Hamming weights are taken in ascending
 *       order w = 1, 2, ... (the union order of eq. (fractionation)); Hamming
 *       weights whose class is empty (W' > w (n - w)) are skipped.
 *   R4  Query 1 is the empty pattern (no flip) and counts as a query.
 *   R5  The budget is the largest number of queries made; with no member found
 *       the decoder returns the hard decision, queries = budget, abandon = 1.
 *   R6  Build-mountain with W'' = 0 sets q = r = 0 (no division needed).
 *
 * Learned-order variant: the patterns are grouped in batches of 64 by global
 * index g (batch b = [64b, 64b+64)); the caller gives a permutation of the
 * first 64 batches, which are tested in that order (ascending g inside a
 * batch), then the plain order continues from g = 4096.  The budget and the
 * abandonment rule are unchanged.
 *
 * 1-line ORBGRAND (the full ORBGRAND of Sec. IV with m = 1 segment): the
 * reliability of rank j is modelled as J0 + beta j (eq. (relest_seg)), so a
 * pattern's reliability weight is J0 w + beta W (eq. (W2IJ)) with w its Hamming
 * and W its logistic weight; patterns are taken by increasing reliability
 * weight, and inside one weight by the rules above.  Fitting and quantization
 * (Sec. IV, eqs. (Q), (quant)) with m = 1:
 *   R10 the anchor points are ranks 1 and h = floor(n/2) and the one line joins
 *       them (the central line extended over the whole curve), so
 *       Q = (L_h - L_1) / (h - 1), beta = [Q / Q] = 1 and J0 = [L_1 / Q] - 1,
 *       L_j the j-th smallest |LLR|; with beta = 1 the weight is J0 w + W;
 *   R11 [x] rounds half up, floor(x + 1/2); the fit runs in FP32 in exactly
 *       this order; Q <= 0, NaN or infinite values give J0 = 0 (basic
 *       ORBGRAND), and J0 is capped at 2^20 (far beyond any weight reached).
 *   With J0 = 0 the order is the basic one.
 *
 * Parity status: every function here is pinned by tests (brute-force
 * enumeration, closed forms, the paper's worked partition example and first
 * queries, brute-force ML over all codewords of tiny codes).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <limits.h>

#define ORACLE_NMAX 1024

/* ------------------------------------------------------------------------ */
/* Build-mountain and Landslide (Sec. III-C, Algorithm 2).                   */
/* Parts are 1-based: u[1..w]; u[0] is the dummy part equal to 0 used for    */
/* the initial mountain.                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int Wp;          /* W' : integer to partition                            */
    int w;           /* number of parts                                       */
    int np;          /* n' : largest allowed part                             */
    int u[ORACLE_NMAX + 1];
    int started;     /* first partition emitted?                              */
    int finished;
} landslide_t;

/* Build-mountain from part k (0 <= k <= w): the parts after k are first set
 * equal to u_k, then the unallocated cells are pushed to the right-most parts,
 * each capped at n'.  Returns 0 on success, -1 if the cells cannot be placed
 * (the caller only asks for feasible classes, so this signals a bug). */
static int build_mountain(landslide_t* s, int k)
{
    int w = s->w, np = s->np;
    int i;
    long sum = 0, Wpp, q, r, room;
    for (i = k + 1; i <= w; ++i) s->u[i] = s->u[k];          /* step 1 */
    for (i = 1; i <= w; ++i) sum += s->u[i];
    Wpp = (long)s->Wp - sum;                                  /* step 2 */
    if (Wpp < 0) return -1;
    room = (long)np - s->u[k];
    if (Wpp == 0) { q = 0; r = 0; }                           /* reading R6 */
    else {
        if (room <= 0) return -1;
        q = Wpp / room; r = Wpp % room;                       /* step 3 */
    }
    if (q > w - k) return -1;
    if (q != 0)
        for (i = w - (int)q + 1; i <= w; ++i) s->u[i] = np;   /* step 4 */
    s->u[w - q] += (int)r;                                    /* step 5 */
    if (w - q == k && r != 0 && k >= 1) return -1;            /* would alter a fixed part */
    if (s->u[w - q] > np) return -1;
    return 0;
}

/* Accumulated drop D(i) = sum_{j>=i} d(j) with d(j) = u_{j+1} - u_j and
 * d(w) = 0, i.e. D(i) = u_w - u_i. */
static int acc_drop(const landslide_t* s, int i)
{
    int j, D = 0;
    for (j = i; j <= s->w; ++j) D += (j == s->w) ? 0 : (s->u[j + 1] - s->u[j]);
    return D;
}

/* Returns 1 if the class (W', w, n') is non-empty and the generator is ready. */
static int landslide_init(landslide_t* s, int Wp, int w, int np)
{
    memset(s, 0, sizeof(*s));
    s->Wp = Wp; s->w = w; s->np = np;
    if (w < 1 || w > ORACLE_NMAX || np < 0 || Wp < 0) return 0;
    if ((long)Wp > (long)w * np) return 0;
    return 1;
}

/* Emit the next partition into out[0..w-1] (u_1..u_w); returns 0 when done. */
static int landslide_next(landslide_t* s, int* out)
{
    int i, k;
    if (s->finished) return 0;
    if (!s->started) {
        s->u[0] = 0;                                   /* dummy part u_0 = 0 */
        if (build_mountain(s, 0) != 0) { s->finished = 1; return 0; }
        s->started = 1;
    } else {
        if (acc_drop(s, 1) < 2) { s->finished = 1; return 0; }
        k = 0;
        for (i = s->w; i >= 1; --i)
            if (acc_drop(s, i) >= 2) { k = i; break; }  /* largest k, D(k) >= 2 */
        s->u[k] += 1;
        if (build_mountain(s, k) != 0) { s->finished = 1; return 0; }
    }
    for (i = 1; i <= s->w; ++i) out[i - 1] = s->u[i];
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Canonical basic-ORBGRAND query order (Sec. III-B): W ascending, then w     */
/* ascending (reading R3), then Landslide order inside (W, w).  Patterns are  */
/* given as 1-based reliability ranks v_1 < ... < v_w.                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;
    long W;          /* current logistic weight                             */
    int w;           /* current Hamming weight                              */
    long Wmax;       /* n(n+1)/2                                            */
    int empty_done;  /* the W = 0 pattern has been emitted                   */
    int active;      /* a Landslide generator is running for (W, w)         */
    landslide_t ls;
} orb_order_t;

static void order_init(orb_order_t* o, int n)
{
    memset(o, 0, sizeof(*o));
    o->n = n;
    o->Wmax = (long)n * (n + 1) / 2;
    o->W = 0;
    o->w = 0;
}

/* Largest Hamming weight allowed by eq. (fractionation): floor((sqrt(1+8W)-1)/2),
 * computed in integers as the largest w with w(w+1)/2 <= W. */
static int max_hamming(long W)
{
    int w = 0;
    while ((long)(w + 1) * (w + 2) / 2 <= W) ++w;
    return w;
}

/* Next pattern in the order: writes ranks to v[0..*w-1]; returns 0 when all
 * 2^n patterns have been produced. */
static int order_next(orb_order_t* o, int* v, int* wout)
{
    int u[ORACLE_NMAX];
    int i;
    if (!o->empty_done) { o->empty_done = 1; *wout = 0; return 1; }
    for (;;) {
        if (o->active && landslide_next(&o->ls, u)) {
            for (i = 0; i < o->w; ++i) v[i] = u[i] + i + 1;   /* eq. (vu) */
            *wout = o->w;
            return 1;
        }
        o->active = 0;
        /* advance (W, w) */
        if (o->W == 0) { o->W = 1; o->w = 0; }
        o->w += 1;
        while (o->w > max_hamming(o->W) || o->w > o->n) {
            o->W += 1; o->w = 1;
            if (o->W > o->Wmax) return 0;
        }
        {
            long Wp = o->W - (long)o->w * (o->w + 1) / 2;     /* W' */
            int np = o->n - o->w;                              /* n' */
            if (Wp <= (long)o->w * np &&
                landslide_init(&o->ls, (int)Wp, o->w, np))
                o->active = 1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* 1-line order: classes (W, w) taken by increasing J0 w + W, then w.         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;
    long J0;
    long C;          /* current reliability weight J0 w + W                  */
    int w;           /* current Hamming weight                              */
    int empty_done;
    int active;
    landslide_t ls;
} orb1_order_t;

/* Smallest and largest logistic weight of w distinct ranks in [1, n]. */
static long lw_min(int w) { return (long)w * (w + 1) / 2; }
static long lw_max(int w, int n) { return (long)w * n - (long)w * (w - 1) / 2; }

static void order1_init(orb1_order_t* o, int n, long J0)
{
    memset(o, 0, sizeof(*o));
    o->n = n;
    o->J0 = J0;
    o->C = 0;
    o->w = 0;
}

/* Next pattern of the 1-line order (same output convention as order_next). */
static int order1_next(orb1_order_t* o, int* v, int* wout)
{
    int u[ORACLE_NMAX];
    int i;
    if (!o->empty_done) { o->empty_done = 1; *wout = 0; return 1; }   /* weight 0, w = 0 first */
    for (;;) {
        if (o->active && landslide_next(&o->ls, u)) {
            for (i = 0; i < o->w; ++i) v[i] = u[i] + i + 1;
            *wout = o->w;
            return 1;
        }
        o->active = 0;
        /* advance (C, w): w ascending while some w can still reach C */
        for (;;) {
            o->w += 1;
            if (o->w <= o->n && lw_min(o->w) + o->J0 * o->w <= o->C) break;
            /* no larger w at this weight: next weight that some w can reach */
            {
                long next = -1;
                int ww;
                for (ww = 1; ww <= o->n; ++ww) {
                    long lo = o->J0 * ww + lw_min(ww), hi = o->J0 * ww + lw_max(ww, o->n);
                    long c = (o->C + 1 > lo) ? o->C + 1 : lo;
                    if (c <= hi && (next < 0 || c < next)) next = c;
                }
                if (next < 0) return 0;                 /* all 2^n patterns done */
                o->C = next;
                o->w = 0;
            }
        }
        {
            long W = o->C - o->J0 * o->w;              /* logistic weight of the class */
            long Wp = W - lw_min(o->w);
            int np = o->n - o->w;
            if (Wp >= 0 && Wp <= (long)o->w * np && landslide_init(&o->ls, (int)Wp, o->w, np))
                o->active = 1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Exported helpers for the tests.                                            */
/* ------------------------------------------------------------------------ */

/* All partitions of W' into w non-decreasing parts in [0, n'], in Landslide
 * order; out holds max_count rows of w ints.  Returns the number produced
 * (or the total count if out is NULL). */
long oracle_landslide(int Wp, int w, int np, int* out, long max_count)
{
    landslide_t s;
    int u[ORACLE_NMAX];
    long c = 0;
    int i;
    if (!landslide_init(&s, Wp, w, np)) return 0;
    while (landslide_next(&s, u)) {
        if (out && c < max_count)
            for (i = 0; i < w; ++i) out[c * w + i] = u[i];
        ++c;
        if (out && c >= max_count) break;
    }
    return c;
}

/* First `count` patterns of the order for length n.  Row g of out holds
 * `width` ints: the ranks v_1..v_w followed by zeros; wout[g] = w.  Returns
 * the number of rows produced (less than count once all 2^n are done), or -1
 * if a pattern is wider than `width`. */
long oracle_order_prefix(int n, long count, int width, int* out, int* wout)
{
    orb_order_t* o = (orb_order_t*)malloc(sizeof(orb_order_t));
    int v[ORACLE_NMAX];
    int w, i;
    long g = 0;
    if (!o) return -2;
    order_init(o, n);
    while (g < count && order_next(o, v, &w)) {
        if (w > width) { free(o); return -1; }
        for (i = 0; i < width; ++i) out[g * width + i] = (i < w) ? v[i] : 0;
        wout[g] = w;
        ++g;
    }
    free(o);
    return g;
}

/* ------------------------------------------------------------------------ */
/* Decoder (Algorithm 1 with the basic ORBGRAND generator).                   */
/* ------------------------------------------------------------------------ */

static uint64_t sort_key(float x, int i)
{
    uint32_t b;
    float a = fabsf(x);
    memcpy(&b, &a, 4);
    return ((uint64_t)b << 32) | (uint32_t)i;
}

/* pi[j] = received index of the (j+1)-th least reliable bit (reading R2);
 * a plain insertion sort on the keys. */
static void reliability_permutation(const float* llr, int n, int* pi)
{
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    int i, j;
    for (i = 0; i < n; ++i) key[i] = sort_key(llr[i], i);
    for (i = 1; i < n; ++i) {
        uint64_t k = key[i];
        j = i - 1;
        while (j >= 0 && key[j] > k) { key[j + 1] = key[j]; --j; }
        key[j + 1] = k;
    }
    for (i = 0; i < n; ++i) pi[i] = (int)(key[i] & 0xffffffffu);
    free(key);
}

/* Code-book membership: is H x = 0 over GF(2)?  H is (n-k) x n, row-major. */
static int in_codebook(const uint8_t* H, int m, int n, const uint8_t* x)
{
    int r, i;
    for (r = 0; r < m; ++r) {
        int acc = 0;
        for (i = 0; i < n; ++i) acc ^= (H[(size_t)r * n + i] & x[i]);
        if (acc & 1) return 0;
    }
    return 1;
}

static int check_args(const uint8_t* H, const float* llr, int n, int k, uint64_t budget)
{
    int i;
    if (!H || !llr) return -1;
    if (n < 1 || n > ORACLE_NMAX || k < 0 || k >= n || budget == 0) return -1;
    for (i = 0; i < (n - k) * n; ++i) if (H[i] > 1) return -1;
    return 0;
}

/* Decode one block.  `order` is NULL for plain ORBGRAND, or a permutation of
 * 0..63 giving the test order of the first 64 batches of 64 patterns. */
static int decode_one(const uint8_t* H, const float* llr, int n, int k,
                      uint64_t budget, const uint8_t* order,
                      uint8_t* cw, uint64_t* queries, uint8_t* abandoned)
{
    int m = n - k;
    int i, w;
    int v[ORACLE_NMAX];
    int* pi = (int*)malloc(sizeof(int) * (size_t)n);
    uint8_t* y = (uint8_t*)malloc((size_t)n);
    uint8_t* x = (uint8_t*)malloc((size_t)n);
    uint64_t q = 0;
    int found = 0;

    for (i = 0; i < n; ++i) y[i] = (llr[i] > 0.0f) ? 1 : 0;   /* reading R1 */
    reliability_permutation(llr, n, pi);

    if (!order) {
        orb_order_t* o = (orb_order_t*)malloc(sizeof(orb_order_t));
        order_init(o, n);
        while (q < budget && order_next(o, v, &w)) {
            ++q;
            memcpy(x, y, (size_t)n);
            for (i = 0; i < w; ++i) x[pi[v[i] - 1]] ^= 1;
            if (in_codebook(H, m, n, x)) { found = 1; break; }
        }
        free(o);
    } else {
        /* Materialise the 4096-pattern prefix, then test it batch by batch in
         * the given order; afterwards continue the plain order. */
        int* pre = (int*)malloc(sizeof(int) * 4096 * 16);
        int* prew = (int*)malloc(sizeof(int) * 4096);
        orb_order_t* o = (orb_order_t*)malloc(sizeof(orb_order_t));
        int t, l, have = 0;
        order_init(o, n);
        while (have < 4096 && order_next(o, v, &w)) {
            for (i = 0; i < 16; ++i) pre[have * 16 + i] = (i < w) ? v[i] : 0;
            prew[have] = w;
            ++have;
        }
        for (t = 0; t < 64 && !found && q < budget; ++t) {
            int b = order[t];
            for (l = 0; l < 64 && q < budget; ++l) {
                int g = b * 64 + l;
                if (g >= have) break;
                ++q;
                memcpy(x, y, (size_t)n);
                for (i = 0; i < prew[g]; ++i) x[pi[pre[g * 16 + i] - 1]] ^= 1;
                if (in_codebook(H, m, n, x)) { found = 1; break; }
            }
        }
        /* the generator already stands at g = 4096 (or is exhausted) */
        while (!found && q < budget && have == 4096 && order_next(o, v, &w)) {
            ++q;
            memcpy(x, y, (size_t)n);
            for (i = 0; i < w; ++i) x[pi[v[i] - 1]] ^= 1;
            if (in_codebook(H, m, n, x)) { found = 1; break; }
        }
        free(o); free(pre); free(prew);
    }

    if (found) {
        memcpy(cw, x, (size_t)n);
        *queries = q;
        *abandoned = 0;
    } else {                                                  /* reading R5 */
        memcpy(cw, y, (size_t)n);
        *queries = budget;
        *abandoned = 1;
    }
    free(pi); free(y); free(x);
    return 0;
}

/* Decode `batch` blocks of one code.  llr is batch x n row-major, cw is
 * batch x n bytes (0/1), queries and abandoned have one entry per block.
 * `threads` > 1 decodes blocks in parallel (independent blocks; OpenMP). */
int oracle_decode(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                  long batch, uint8_t* cw, uint64_t* queries, uint8_t* abandoned,
                  int threads)
{
    long b;
    if (check_args(H, llr, n, k, budget) != 0 || batch < 0) return -1;
    (void)threads;
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
    for (b = 0; b < batch; ++b)
        decode_one(H, llr + (size_t)b * n, n, k, budget, NULL,
                   cw + (size_t)b * n, queries + b, abandoned + b);
    return 0;
}

/* Learned-order decode: order is batch x 64 bytes, each row a permutation of
 * 0..63.  Requires n >= 12 so that the first 4096 patterns exist. */
int oracle_decode_ordered(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                          long batch, const uint8_t* order, uint8_t* cw,
                          uint64_t* queries, uint8_t* abandoned, int threads)
{
    long b;
    if (check_args(H, llr, n, k, budget) != 0 || batch < 0 || !order || n < 12) return -1;
    for (b = 0; b < batch; ++b) {
        int seen[64] = {0}, t;
        for (t = 0; t < 64; ++t) {
            int o = order[b * 64 + t];
            if (o > 63 || seen[o]) return -1;
            seen[o] = 1;
        }
    }
    (void)threads;
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
    for (b = 0; b < batch; ++b)
        decode_one(H, llr + (size_t)b * n, n, k, budget, order + (size_t)b * 64,
                   cw + (size_t)b * n, queries + b, abandoned + b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 1-line ORBGRAND decoder.                                                   */
/* ------------------------------------------------------------------------ */

/* J0 of one block from its reliability order (readings R10, R11). */
static long fit_j0(const float* llr, const int* pi, int n)
{
    int h = n / 2;
    float L1, Lh, Q, r;
    if (h < 2) return 0;
    L1 = fabsf(llr[pi[0]]);
    Lh = fabsf(llr[pi[h - 1]]);
    Q = (Lh - L1) / (float)(h - 1);
    if (!(Q > 0.0f) || !isfinite(Q)) return 0;
    r = L1 / Q;
    if (!isfinite(r)) return 0;
    r = floorf(r + 0.5f);
    if (r > 1048576.0f) r = 1048576.0f;
    return (long)r - 1;
}

static int decode_one_1line(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                            long j0_force, uint8_t* cw, uint64_t* queries, uint8_t* abandoned,
                            int32_t* j0_out)
{
    int m = n - k;
    int i, w;
    int v[ORACLE_NMAX];
    int* pi = (int*)malloc(sizeof(int) * (size_t)n);
    uint8_t* y = (uint8_t*)malloc((size_t)n);
    uint8_t* x = (uint8_t*)malloc((size_t)n);
    orb1_order_t* o = (orb1_order_t*)malloc(sizeof(orb1_order_t));
    uint64_t q = 0;
    int found = 0;
    long J0;

    for (i = 0; i < n; ++i) y[i] = (llr[i] > 0.0f) ? 1 : 0;
    reliability_permutation(llr, n, pi);
    J0 = (j0_force != LONG_MIN) ? j0_force : fit_j0(llr, pi, n);
    if (j0_out) *j0_out = (int32_t)J0;
    order1_init(o, n, J0);
    while (q < budget && order1_next(o, v, &w)) {
        ++q;
        memcpy(x, y, (size_t)n);
        for (i = 0; i < w; ++i) x[pi[v[i] - 1]] ^= 1;
        if (in_codebook(H, m, n, x)) { found = 1; break; }
    }
    if (found) {
        memcpy(cw, x, (size_t)n);
        *queries = q;
        *abandoned = 0;
    } else {
        memcpy(cw, y, (size_t)n);
        *queries = budget;
        *abandoned = 1;
    }
    free(o); free(pi); free(y); free(x);
    return 0;
}

/* 1-line decode of `batch` blocks (layout as oracle_decode).  j0_out (may be
 * NULL) receives each block's J0; j0_force != LONG_MIN replaces the fit by
 * that value for every block (tests of the order alone). */
int oracle_decode_1line(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, long batch,
                        uint8_t* cw, uint64_t* queries, uint8_t* abandoned, int32_t* j0_out,
                        long j0_force, int threads)
{
    long b;
    if (check_args(H, llr, n, k, budget) != 0 || batch < 0) return -1;
    if (j0_force != LONG_MIN && (j0_force < -1 || j0_force > 1048575)) return -1;
    (void)threads;
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
    for (b = 0; b < batch; ++b)
        decode_one_1line(H, llr + (size_t)b * n, n, k, budget, j0_force, cw + (size_t)b * n,
                         queries + b, abandoned + b, j0_out ? j0_out + b : NULL);
    return 0;
}

/* First `count` patterns of the 1-line order for (n, J0), as oracle_order_prefix. */
long oracle_order1_prefix(int n, long j0, long count, int width, int* out, int* wout)
{
    orb1_order_t* o = (orb1_order_t*)malloc(sizeof(orb1_order_t));
    int v[ORACLE_NMAX];
    int w, i;
    long g = 0;
    if (!o) return -2;
    order1_init(o, n, j0);
    while (g < count && order1_next(o, v, &w)) {
        if (w > width) { free(o); return -1; }
        for (i = 0; i < width; ++i) out[g * width + i] = (i < w) ? v[i] : 0;
        wout[g] = w;
        ++g;
    }
    free(o);
    return g;
}

/* The 1-line fit alone: J0 of one block. */
long oracle_fit_j0(const float* llr, int n)
{
    int* pi = (int*)malloc(sizeof(int) * (size_t)n);
    long j0;
    reliability_permutation(llr, n, pi);
    j0 = fit_j0(llr, pi, n);
    free(pi);
    return j0;
}

/* Syndrome-free membership test exposed for the invariant tests. */
int oracle_is_codeword(const uint8_t* H, int n, int k, const uint8_t* x)
{
    return in_codebook(H, n - k, n, x);
}

/* Reliability permutation exposed for the tests (pi is 0-based indices). */
void oracle_permutation(const float* llr, int n, int* pi)
{
    reliability_permutation(llr, n, pi);
}
