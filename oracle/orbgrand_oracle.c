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
 * 1-line ORBGRAND (the full ORBGRAND of Sec. III-D with m = 1 segment): the
 * reliability of rank j is modelled as J0 + beta j (eq. (relest_seg)), so a
 * pattern's reliability weight is J0 w + beta W (eq. (W2IJ)) with w its Hamming
 * and W its logistic weight; patterns are taken by increasing reliability
 * weight, and inside one weight by the rules above.  Fitting and quantization
 * (Sec. III-E, eqs. (Q), (quant)) with m = 1:
 *   R10 the anchor points are ranks 1 and h = floor(n/2) and the one line joins
 *       them (the central line extended over the whole curve), so
 *       Q = (L_h - L_1) / (h - 1), beta = [Q / Q] = 1 and J0 = [L_1 / Q] - 1,
 *       L_j the j-th smallest |LLR|; with beta = 1 the weight is J0 w + W;
 *   R11 [x] rounds half up, floor(x + 1/2); the fit runs in FP32 in exactly
 *       this order; Q <= 0, NaN or infinite values give J0 = 0 (basic
 *       ORBGRAND), and J0 is capped at 2^20 (far beyond any weight reached).
 *   With J0 = 0 the order is the basic one.
 *
 * Full ORBGRAND (Sec. III-D with m segments, the fit of eqs. (Q), (quant) and the
 * J/beta variant) follows at the end of the file with readings R12-R15.
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

/* ------------------------------------------------------------------------ */
/* Full (m-line) ORBGRAND, Sec. III-D.                                          */
/*                                                                            */
/* Model (eq. (relest_seg)): segment i (1 <= i <= m) holds ranks              */
/* I[i-1]+1 .. I[i], I[0] = 0, I[m] = n, and models the reliability of rank j */
/* as J[i-1] + beta[i-1] (j - I[i-1]).  A pattern's reliability weight is the */
/* sum over segments of J[i-1] w_i + beta[i-1] W'_i (eq. (W2IJ)), w_i and W'_i */
/* the Hamming weight and the logistic weight of its ranks in segment i,      */
/* counted from the segment's start.                                          */
/*                                                                            */
/* Order (eq. (cartP) and the flow of Sec. III-D): reliability weights W          */
/* ascending; inside one W, the splitting patterns (W_1, ..., W_m),           */
/* sum W, in the nested-loop order of the integer splitting algorithm (W_1    */
/* ascending, then W_2, ...), only those whose every W_i has a valid partial  */
/* Hamming weight (the collection algorithm); inside one split the Cartesian  */
/* product of the partial sets, segment 1 outermost; a partial set is the     */
/* union over valid partial Hamming weights w ascending of the Landslide      */
/* sequence of that (w, W'_i) in the segment.                                  */
/*                                                                            */
/* Readings (also in the design notes):                                       */
/*   R12 validity of (W_i, w) in segment i: the empty partial pattern (w = 0) */
/*       has W_i = 0; for w >= 1, W_i - w J[i-1] divisible by beta[i-1] and   */
/*       the quotient W' between w(w+1)/2 and w n_i - w(w-1)/2, n_i the       */
/*       segment length (the bounds of eq. (wi_cond) with the factor beta of  */
/*       eq. (wu_i) restored, taken as the whole condition).  Every w meeting */
/*       it counts: the collection algorithm's upper loop bound on w holds    */
/*       only for J >= 0, and with J0 < 0 (down to -beta_1) a weight can have */
/*       more flips than that bound allows (rank 1 alone weighs 0 at          */
/*       J0 = -beta_1).                                                       */
/*   R13 ties inside one partial set: w ascending (as R3), Landslide order   */
/*       inside one w; the Cartesian product runs with segment 1 outermost.  */
/*   R14 anchors: ranks 1 and h = floor(n/2) first; each further anchor is    */
/*       the rank with the largest vertical gap |L_j - line_j| between the    */
/*       curve and the chord of the two adjacent anchors around it, over all  */
/*       adjacent pairs (smallest j on ties); no anchor is added when the     */
/*       largest gap is 0 or none is left, so fewer segments may result.     */
/*       The chord at j is L_a + (j - a) s with s = (L_b - L_a)/(b - a), in   */
/*       FP32 in that order.  Segments: I[i] = anchor i for 1 <= i <= m-1, the */
/*       last segment extended to n (the central line covers the rest).       */
/*   R15 quantization (eqs. (Q), (quant)) in FP32 with the anchors as I:      */
/*       slope_1 = (L_a1 - L_1)/(a1 - 1), slope_i = (L_ai - L_a(i-1))/(ai -    */
/*       a(i-1)); Q = the smallest slope; beta_i = [d_i / (len_i Q)] with d_i */
/*       and len_i the slope's numerator and denominator (the product first), */
/*       J0 = [L_1/Q] - beta_1, J_i = [L_ai/Q]; [x] = floor(x + 1/2), capped  */
/*       at 2^20.  Q not positive and finite, or any value not finite, gives  */
/*       the basic model (m = 1, J0 = 0, beta = 1).  With one segment this is  */
/*       the 1-line fit (R10).                                                 */
/* ------------------------------------------------------------------------ */

#define ORBM_MMAX 8

typedef struct {
    int m;
    int I[ORBM_MMAX + 1];
    long J[ORBM_MMAX];
    long beta[ORBM_MMAX];
} orbm_model_t;

static void model_basic(orbm_model_t* M, int n)
{
    memset(M, 0, sizeof(*M));
    M->m = 1;
    M->I[0] = 0;
    M->I[1] = n;
    M->J[0] = 0;
    M->beta[0] = 1;
}

static int round_half_up(float x, long* out)
{
    float r;
    if (!isfinite(x)) return -1;
    r = floorf(x + 0.5f);
    if (r > 1048576.0f) r = 1048576.0f;
    *out = (long)r;
    return 0;
}

/* Model of one block with at most mreq segments (readings R14, R15). */
static void fit_mline(const float* llr, const int* pi, int n, int mreq, orbm_model_t* M)
{
    int h = n / 2, na = 2, it, i, j, p;
    int a[ORBM_MMAX + 1];
    float* L;
    float Q = 0.0f;
    float d[ORBM_MMAX], len[ORBM_MMAX];
    model_basic(M, n);
    if (h < 2 || mreq < 1) return;
    if (mreq > ORBM_MMAX) mreq = ORBM_MMAX;
    L = (float*)malloc(sizeof(float) * (size_t)(h + 1));
    for (j = 1; j <= h; ++j) L[j] = fabsf(llr[pi[j - 1]]);
    a[0] = 1;
    a[1] = h;
    for (it = 1; it < mreq; ++it) {
        float best = -1.0f;
        int bj = 0, bpos = 0;
        for (p = 0; p + 1 < na; ++p) {
            float s;
            if (a[p + 1] - a[p] < 2) continue;
            s = (L[a[p + 1]] - L[a[p]]) / (float)(a[p + 1] - a[p]);
            for (j = a[p] + 1; j < a[p + 1]; ++j) {
                float t = (float)(j - a[p]) * s;
                float line = L[a[p]] + t;
                float gap = fabsf(L[j] - line);
                if (gap > best) { best = gap; bj = j; bpos = p + 1; }
            }
        }
        if (!(best > 0.0f)) break;
        for (p = na; p > bpos; --p) a[p] = a[p - 1];
        a[bpos] = bj;
        ++na;
    }
    {
        int m = na - 1;
        long rb;
        for (i = 0; i < m; ++i) {
            int lo = a[i], hi = a[i + 1];
            d[i] = L[hi] - L[lo];
            len[i] = (float)(hi - lo);
            {
                float s = d[i] / len[i];
                if (i == 0 || s < Q) Q = s;
            }
        }
        if (!(Q > 0.0f) || !isfinite(Q)) { free(L); return; }
        M->m = m;
        M->I[0] = 0;
        for (i = 1; i < m; ++i) M->I[i] = a[i];
        M->I[m] = n;
        for (i = 0; i < m; ++i) {
            float t = len[i] * Q;
            if (round_half_up(d[i] / t, &M->beta[i]) != 0 || M->beta[i] < 1) { model_basic(M, n); free(L); return; }
        }
        if (round_half_up(L[1] / Q, &rb) != 0) { model_basic(M, n); free(L); return; }
        M->J[0] = rb - M->beta[0];
        for (i = 1; i < m; ++i)
            if (round_half_up(L[a[i]] / Q, &M->J[i]) != 0) { model_basic(M, n); free(L); return; }
    }
    free(L);
}

/* Segment i (0-based) of model M: length, offset, slope. */
static int seg_len(const orbm_model_t* M, int i) { return M->I[i + 1] - M->I[i]; }

/* Is W a partial weight of segment i with partial Hamming weight w (R12)?
 * Writes the relative logistic weight. */
static int seg_valid_w(const orbm_model_t* M, int i, long W, int w, long* Wp)
{
    int ni = seg_len(M, i);
    long r;
    if (w == 0) { *Wp = 0; return W == 0; }
    if (w > ni) return 0;
    r = W - (long)w * M->J[i];
    if (r < 0 || r % M->beta[i] != 0) return 0;
    r /= M->beta[i];
    if (r < lw_min(w) || r > lw_max(w, ni)) return 0;
    *Wp = r;
    return 1;
}

/* The collection step: does W have a valid partial Hamming weight in segment i? */
static int seg_valid(const orbm_model_t* M, int i, long W)
{
    int w;
    long Wp;
    for (w = 0; w <= seg_len(M, i); ++w)
        if (seg_valid_w(M, i, W, w, &Wp)) return 1;
    return 0;
}


/* Smallest partial weight of segment i that is >= x (LONG_MAX if none): the
 * next value at which the nested loop of the splitting algorithm finds a
 * valid W_i (the jump over values the collection algorithm would reject). */
static long seg_next(const orbm_model_t* M, int i, long x)
{
    int ni = seg_len(M, i), w;
    long best = LONG_MAX;
    if (x <= 0) return 0;                                  /* the empty partial pattern */
    for (w = 1; w <= ni; ++w) {
        long lo = lw_min(w), hi = lw_max(w, ni), need = x - (long)w * M->J[i], Wp, c;
        Wp = need <= 0 ? lo : (need + M->beta[i] - 1) / M->beta[i];
        if (Wp < lo) Wp = lo;
        if (Wp > hi) continue;
        c = (long)w * M->J[i] + M->beta[i] * Wp;
        if (c < best) best = c;
    }
    return best;
}

/* Largest reliability weight of any pattern of the model. */
static long model_wmax(const orbm_model_t* M)
{
    long t = 0;
    int i, w;
    for (i = 0; i < M->m; ++i) {
        long best = 0;
        for (w = 1; w <= seg_len(M, i); ++w) {
            long c = (long)w * M->J[i] + M->beta[i] * lw_max(w, seg_len(M, i));
            if (c > best) best = c;
        }
        t += best;
    }
    return t;
}

/* reach(i, x): can segments i..m-1 have partial weights summing to exactly x?
 * Memoised per segment (0 unknown, 1 no, 2 yes). */
typedef struct {
    const orbm_model_t* M;
    unsigned char* memo[ORBM_MMAX];
    long size[ORBM_MMAX];
} reach_t;

static int reach(reach_t* R, int i, long x)
{
    const orbm_model_t* M = R->M;
    long a;
    int r = 1;
    if (x < 0) return 0;
    if (i == M->m - 1) return seg_valid(M, i, x);
    if (x >= R->size[i]) {
        long ns = R->size[i] ? R->size[i] : 1024;
        while (ns <= x) ns *= 2;
        R->memo[i] = (unsigned char*)realloc(R->memo[i], (size_t)ns);
        memset(R->memo[i] + R->size[i], 0, (size_t)(ns - R->size[i]));
        R->size[i] = ns;
    }
    if (R->memo[i][x]) return R->memo[i][x] == 2;
    for (a = 0; a <= x; a = seg_next(M, i, a + 1))
        if (reach(R, i + 1, x - a)) { r = 2; break; }
    R->memo[i][x] = (unsigned char)r;
    return r == 2;
}

/* Partial set of segment i for partial weight W (R12, R13): the partial
 * patterns as relative ranks, w ascending, Landslide order inside.  Stored
 * flat: pattern p has ranks flat[start[p] .. start[p] + w[p]). */
typedef struct { int* flat; long* start; int* w; long count, cap, used, fcap; } pset_t;

static void pset_push(pset_t* s, const int* v, int w)
{
    int k;
    if (s->count == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 64;
        s->start = (long*)realloc(s->start, sizeof(long) * (size_t)s->cap);
        s->w = (int*)realloc(s->w, sizeof(int) * (size_t)s->cap);
    }
    while (s->used + w > s->fcap) {
        s->fcap = s->fcap ? 2 * s->fcap : 256;
        s->flat = (int*)realloc(s->flat, sizeof(int) * (size_t)s->fcap);
    }
    for (k = 0; k < w; ++k) s->flat[s->used + k] = v[k];
    s->start[s->count] = s->used;
    s->w[s->count++] = w;
    s->used += w;
}

static void pset_build(const orbm_model_t* M, int i, long W, pset_t* s)
{
    int ni = seg_len(M, i), w, k;
    int* u = (int*)malloc(sizeof(int) * (size_t)(ni + 1));
    int* v = (int*)malloc(sizeof(int) * (size_t)(ni + 1));
    landslide_t* ls = (landslide_t*)malloc(sizeof(landslide_t));
    long Wp;
    s->count = 0;
    s->used = 0;
    for (w = 0; w <= ni; ++w) {
        if (!seg_valid_w(M, i, W, w, &Wp)) continue;
        if (w == 0) { pset_push(s, v, 0); continue; }
        if (!landslide_init(ls, (int)(Wp - lw_min(w)), w, ni - w)) continue;   /* eq. (intpart2) */
        while (landslide_next(ls, u)) {
            for (k = 0; k < w; ++k) v[k] = u[k] + k + 1;                       /* eq. (vu) */
            pset_push(s, v, w);
        }
    }
    free(u); free(v); free(ls);
}

/* The m-line order as a generator driven by callbacks: emit(ranks, w, ctx) is
 * called per pattern (absolute 1-based ranks, ascending inside each segment)
 * and stops the walk by returning nonzero. */
typedef int (*emit_fn)(const int* ranks, int w, void* ctx);

typedef struct {
    const orbm_model_t* M;
    reach_t R;
    long split[ORBM_MMAX];
    pset_t sets[ORBM_MMAX];
    int* ranks;
    long count, limit;
    emit_fn emit;
    void* ctx;
    int stop;
} mwalk_t;

/* Cartesian product of the partial sets of the current split, segment 1
 * outermost (eq. (cartP), reading R13). */
static void walk_product(mwalk_t* s)
{
    const orbm_model_t* M = s->M;
    long idx[ORBM_MMAX];
    int i, k;
    for (i = 0; i < M->m; ++i) {
        pset_build(M, i, s->split[i], &s->sets[i]);
        if (s->sets[i].count == 0) return;     /* cannot happen for a valid split */
        idx[i] = 0;
    }
    for (;;) {
        int w = 0;
        if (s->count >= s->limit) { s->stop = 1; return; }
        for (i = 0; i < M->m; ++i) {
            const pset_t* p = &s->sets[i];
            for (k = 0; k < p->w[idx[i]]; ++k) s->ranks[w++] = M->I[i] + p->flat[p->start[idx[i]] + k];
        }
        ++s->count;
        if (s->emit(s->ranks, w, s->ctx)) { s->stop = 1; return; }
        for (i = M->m - 1; i >= 0; --i) {
            if (++idx[i] < s->sets[i].count) break;
            idx[i] = 0;
        }
        if (i < 0) return;
    }
}

/* Splits of `rest` over segments i..m-1 in the nested-loop order of the
 * integer splitting algorithm, keeping only values with a valid partial
 * Hamming weight (the collection algorithm) whose remainder the later
 * segments can still reach. */
static void walk_splits(mwalk_t* s, int i, long rest)
{
    const orbm_model_t* M = s->M;
    long a;
    if (i == M->m - 1) {
        if (seg_valid(M, i, rest)) { s->split[i] = rest; walk_product(s); }
        return;
    }
    for (a = 0; a <= rest && !s->stop; a = seg_next(M, i, a + 1)) {
        if (!reach(&s->R, i + 1, rest - a)) continue;
        s->split[i] = a;
        walk_splits(s, i + 1, rest - a);
    }
}

/* Walks the order of model M for at most `limit` patterns; returns the count. */
static long mline_walk(const orbm_model_t* M, long limit, emit_fn emit, void* ctx)
{
    mwalk_t* s = (mwalk_t*)calloc(1, sizeof(mwalk_t));
    long W, wmax = model_wmax(M), count;
    int i;
    s->M = M;
    s->R.M = M;
    s->ranks = (int*)malloc(sizeof(int) * (size_t)(M->I[M->m] + 1));
    s->limit = limit;
    s->emit = emit;
    s->ctx = ctx;
    for (W = 0; W <= wmax && !s->stop && s->count < limit; ++W)   /* weights ascending */
        if (reach(&s->R, 0, W)) walk_splits(s, 0, W);
    count = s->count;
    for (i = 0; i < ORBM_MMAX; ++i) {
        free(s->sets[i].flat); free(s->sets[i].start); free(s->sets[i].w);
        free(s->R.memo[i]);
    }
    free(s->ranks);
    free(s);
    return count;
}

/* A model given by the caller: m segments, I[0..m] with I[0] = 0 < I[1] <
 * ... < I[m] = n, beta[i] >= 1 and J[i] >= -beta[i] (every pattern weight is
 * then non-negative).  Returns 0 and fills M, or -1. */
static int model_from(int n, int m, const int* I, const long* J, const long* beta, orbm_model_t* M)
{
    int i;
    if (n < 1 || n > ORACLE_NMAX || m < 1 || m > ORBM_MMAX || !I || !J || !beta) return -1;
    if (I[0] != 0 || I[m] != n) return -1;
    for (i = 0; i < m; ++i) {
        if (I[i + 1] <= I[i] || beta[i] < 1 || beta[i] > 1048576 || J[i] < -beta[i] || J[i] > 1048576)
            return -1;
    }
    memset(M, 0, sizeof(*M));
    M->m = m;
    for (i = 0; i <= m; ++i) M->I[i] = I[i];
    for (i = 0; i < m; ++i) { M->J[i] = J[i]; M->beta[i] = beta[i]; }
    return 0;
}

/* J/beta variant (complexity control of Sec. III-D, rounding of Sec. III-E): each J_{i-1} replaced by
 * [J_{i-1} / beta_i] beta_i, with [x] = floor(x + 1/2) taken exactly. */
static void model_jdiv(orbm_model_t* M)
{
    int i;
    for (i = 0; i < M->m; ++i) {
        long num = 2 * M->J[i] + M->beta[i], den = 2 * M->beta[i];
        long q = num / den;
        if (num % den != 0 && num < 0) --q;                /* floor division */
        M->J[i] = q * M->beta[i];
    }
}

typedef struct { long g, count; int width; int* out; int* wout; int overflow; } prefix_ctx_t;

static int prefix_emit(const int* ranks, int w, void* vctx)
{
    prefix_ctx_t* c = (prefix_ctx_t*)vctx;
    int i;
    if (w > c->width) { c->overflow = 1; return 1; }
    for (i = 0; i < c->width; ++i) c->out[c->g * c->width + i] = (i < w) ? ranks[i] : 0;
    c->wout[c->g] = w;
    ++c->g;
    return 0;
}

/* First `count` patterns of the m-line order of a given model (layout as
 * oracle_order_prefix).  Returns the number written, -1 if a pattern is
 * wider than `width`, -2 on an invalid model. */
long oracle_order_mline_prefix(int n, int m, const int* I, const long* J, const long* beta,
                               long count, int width, int* out, int* wout)
{
    orbm_model_t M;
    prefix_ctx_t c;
    if (model_from(n, m, I, J, beta, &M) != 0 || count < 0 || width < 1) return -2;
    c.g = 0; c.count = count; c.width = width; c.out = out; c.wout = wout; c.overflow = 0;
    mline_walk(&M, count, prefix_emit, &c);
    return c.overflow ? -1 : c.g;
}

/* Model of one block: the m-line fit (readings R14, R15) with at most mreq
 * segments, then the J/beta rounding when jdiv is set.  Writes m and
 * I[0..m], J[0..m-1], beta[0..m-1] (arrays of ORBM_MMAX + 1 entries). */
int oracle_fit_mline(const float* llr, int n, int mreq, int jdiv, int* m, int* I, long* J, long* beta)
{
    orbm_model_t M;
    int* pi;
    int i;
    if (!llr || n < 1 || n > ORACLE_NMAX || mreq < 1 || mreq > ORBM_MMAX) return -1;
    pi = (int*)malloc(sizeof(int) * (size_t)n);
    reliability_permutation(llr, n, pi);
    fit_mline(llr, pi, n, mreq, &M);
    if (jdiv) model_jdiv(&M);
    free(pi);
    *m = M.m;
    for (i = 0; i <= M.m; ++i) I[i] = M.I[i];
    for (i = 0; i < M.m; ++i) { J[i] = M.J[i]; beta[i] = M.beta[i]; }
    return 0;
}

typedef struct {
    const uint8_t* H;
    int n, m;
    const int* pi;
    const uint8_t* y;
    uint8_t* x;
    int found;
} decode_ctx_t;

static int decode_emit(const int* ranks, int w, void* vctx)
{
    decode_ctx_t* c = (decode_ctx_t*)vctx;
    int i;
    memcpy(c->x, c->y, (size_t)c->n);
    for (i = 0; i < w; ++i) c->x[c->pi[ranks[i] - 1]] ^= 1;
    if (in_codebook(c->H, c->m, c->n, c->x)) { c->found = 1; return 1; }
    return 0;
}

static void decode_one_mline(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                             int mreq, int jdiv, uint8_t* cw, uint64_t* queries, uint8_t* abandoned,
                             int32_t* m_out)
{
    int i;
    int* pi = (int*)malloc(sizeof(int) * (size_t)n);
    uint8_t* y = (uint8_t*)malloc((size_t)n);
    uint8_t* x = (uint8_t*)malloc((size_t)n);
    orbm_model_t M;
    decode_ctx_t c;
    long q;
    for (i = 0; i < n; ++i) y[i] = (llr[i] > 0.0f) ? 1 : 0;
    reliability_permutation(llr, n, pi);
    fit_mline(llr, pi, n, mreq, &M);
    if (jdiv) model_jdiv(&M);
    if (m_out) *m_out = M.m;
    c.H = H; c.n = n; c.m = n - k; c.pi = pi; c.y = y; c.x = x; c.found = 0;
    q = mline_walk(&M, (long)(budget > (uint64_t)LONG_MAX ? LONG_MAX : budget), decode_emit, &c);
    if (c.found) {
        memcpy(cw, x, (size_t)n);
        *queries = (uint64_t)q;
        *abandoned = 0;
    } else {
        memcpy(cw, y, (size_t)n);
        *queries = budget;
        *abandoned = 1;
    }
    free(pi); free(y); free(x);
}

/* m-line decode of `batch` blocks (layout as oracle_decode): each block's
 * model is fitted with at most mreq segments (J/beta rounding when jdiv is
 * set); m_out (may be NULL) receives each block's segment count. */
int oracle_decode_mline(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, long batch,
                        int mreq, int jdiv, uint8_t* cw, uint64_t* queries, uint8_t* abandoned,
                        int32_t* m_out, int threads)
{
    long b;
    if (check_args(H, llr, n, k, budget) != 0 || batch < 0 || mreq < 1 || mreq > ORBM_MMAX) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
    for (b = 0; b < batch; ++b)
        decode_one_mline(H, llr + (size_t)b * n, n, k, budget, mreq, jdiv, cw + (size_t)b * n,
                         queries + b, abandoned + b, m_out ? m_out + b : NULL);
    return 0;
}
