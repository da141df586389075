/*
 * liborbgrand -- basic Ordered Reliability Bits GRAND on AMD Instinct MI355X
 * (gfx950).  C ABI: plain pointers and sizes, no framework types.
 *
 * Method: Duffy, An, Medard, "Ordered Reliability Bits Guessing Random
 * Additive Noise Decoding" (arXiv 2202.13951).
 *
 * Conventions shared by every entry point
 *   - Status: 0 (ORBG_OK) on success, a negative ORBG_E* code otherwise;
 *     orbg_last_error() then returns a message for the calling thread.
 *   - Parity-check matrix H: HOST pointer, (n - k) rows by n columns,
 *     row-major, one byte per entry, each 0 or 1.  1 <= n <= 1024 and
 *     1 <= n - k <= 64.  The library copies and packs it (column i becomes a
 *     64-bit word whose bit r is H[r][i]; row r becomes 64-bit words whose bit
 *     l of word j is H[r][64 j + l]) into a device cache keyed by its contents;
 *     the caller keeps ownership of H.  If H has rank below n - k the
 *     decoder decodes the code H defines (k only sizes H).
 *   - LLRs: DEVICE pointer, `batch` rows of n FP32 values, row-major, the log
 *     ratio log f(Y|1)/f(Y|0) of Sec. III-A (positive means bit 1).  Values are
 *     not checked: NaN and -0 decide bit 0 and sort by their IEEE bits.
 *   - Outputs: DEVICE pointers owned by the caller: codeword (batch rows of n
 *     bytes, 0/1, in received order), queries (one u64 per block: code-book
 *     queries made, the empty pattern counting as the first), abandoned (one
 *     byte per block: 1 if the budget ran out, then queries == budget and the
 *     codeword row is the hard decision).
 *   - budget: the largest number of queries per block, 1 <= budget <= 5 x 10^6
 *     (the abandonment threshold of Sec. IV-A; the 1-line decode takes at most
 *     2^22).  The query schedule holds every pattern of logistic weight <= 99
 *     and those of weight 100 up to {9, ..., 16} (the only pattern flipping
 *     eight ranks above 8): 5,150,463 patterns for n >= 100, at least 5 x 10^6
 *     for n >= 64; a budget for a short code that would need patterns past
 *     them is rejected with ORBG_EINVAL.
 *   - stream: a hipStream_t (NULL = the default stream).  Decodes are
 *     asynchronous on that stream.  The first call for a new H, or for a new
 *     (n, budget) query schedule, allocates device memory and synchronises the
 *     stream once; later calls do neither.
 *   - Calls from several host threads are safe; calls on different streams
 *     are independent.
 */
#ifndef ORBGRAND_H
#define ORBGRAND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORBG_OK 0
#define ORBG_EINVAL (-1)       /* an argument is out of range or a pointer is NULL */
#define ORBG_ENOMEM (-2)       /* a device allocation failed */
#define ORBG_EHIP (-3)         /* a HIP runtime call or kernel launch failed */

/*
 * Launch shape of a decode (the knobs the autotuner sets).  Any field left 0
 * takes the library default (split_steps: -1 takes the default, 0 disables the
 * heavy pass).  Decodes run in two passes: a light pass of persistent
 * one-wave workgroups over all blocks, which gives up on a block after
 * `split_steps` steps of 64 queries, and a heavy pass in which workgroups of
 * `heavy_waves` waves each share one such block, taking its steps in turn.  The
 * decoded result does not depend on these values.
 */
typedef struct orbg_launch_params {
    int workgroups_per_cu;        /* light pass, 1..64 (default 32) */
    int chunk;                    /* blocks taken per work-counter increment, 1..64 (default: about
                                     4 increments per wave, at most 64) */
    int split_steps;              /* -1 = default (64), 0 = no heavy pass, else steps before the split;
                                     an ordered decode moves values below 64 up to 64 */
    int heavy_waves;              /* 4, 8 or 16 (default 8) */
    int heavy_workgroups_per_cu;  /* heavy pass, 1..16 (default 2) */
    int one_block_per_workgroup;  /* 1: the naive launch -- one one-wave workgroup per block, no work
                                     counter, no chunks, no heavy pass (other fields ignored); 0: the
                                     persistent launch described above */
} orbg_launch_params;

/*
 * Plain basic-ORBGRAND decode of `batch` blocks of one linear code.
 *
 * Follows Algorithm 1 (GRAND: test putative noise patterns from most to least
 * likely; the first y XOR z in the code-book is the decoding) with the basic
 * ORBGRAND pattern order: bits ranked by increasing reliability |LLR| (ties by
 * lower received index), patterns taken by increasing logistic weight (the sum
 * of the flipped ranks, Sec. III-B eq. (lw)), inside one logistic weight by
 * increasing Hamming weight (eq. (fractionation)), inside one (logistic,
 * Hamming) weight in the order of the Landslide generator (Sec. III-C,
 * Algorithm 2).  Membership is the parity-check product H x = 0 (Sec. I).  A
 * block is abandoned once `budget` queries find no member (Sec. IV-A).
 */
int orbg_decode(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                int64_t batch, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned,
                void* stream);

/*
 * Decode with a per-block reordering of the first 4096 patterns.
 *
 * The basic-ORBGRAND order (as in orbg_decode) is cut into batches of 64
 * consecutive patterns; batch b holds global indices [64b, 64b + 64).
 * `order` is a DEVICE array of batch x 64 bytes; row j must be a permutation
 * of 0..63 and gives the order in which block j tests batches 0..63 (ascending
 * index inside a batch).  The plain order then continues from index 4096.
 * `queries` counts positions in this sequence; budget and abandonment are as
 * in orbg_decode.  Requires n >= 12.  Bytes are taken modulo 64; a row that
 * is not a permutation repeats some batches and skips others (the library does
 * not read device memory to check it).
 * This is the decode step of the learned proposal: ORBGRAND's own order stays
 * the fallback after the reordered prefix.
 */
int orbg_decode_ordered(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                        int64_t batch, const uint8_t* order, uint8_t* codeword,
                        uint64_t* queries, uint8_t* abandoned, void* stream);

/*
 * orbg_decode / orbg_decode_ordered with an explicit launch shape.  `order` may
 * be NULL (plain order) or as in orbg_decode_ordered; `params` may be NULL
 * (defaults).  Results are identical for every valid `params`.
 */
int orbg_decode_ex(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                   int64_t batch, const uint8_t* order, uint8_t* codeword, uint64_t* queries,
                   uint8_t* abandoned, const orbg_launch_params* params, void* stream);

/*
 * 1-line ORBGRAND decode (the one-segment case of the full ORBGRAND model of
 * Sec. III-D, noted in Sec. IV-A as giving a small gain over the basic order).
 *
 * Each block's reliability curve is fitted with one line through its anchors at
 * ranks 1 and h = floor(n / 2) (Sec. III-E, anchor-point fitting): slope
 * Q = (L_h - L_1) / (h - 1), with L_j the |LLR| of rank j; quantised offset
 * J0 = [L_1 / Q] - 1, [x] = floor(x + 1/2) (eqs. (Q) and (quant) with m = 1,
 * beta = 1); each operation is FP32 rounded to nearest in that order.  A slope
 * that is not positive and finite, or a ratio L_1 / Q that is not finite, gives
 * J0 = 0, the basic order; [L_1 / Q] is capped at 2^20.  Patterns are then
 * tested by increasing reliability weight J0 w + W (eq. (W2IJ): w Hamming
 * weight, W logistic weight), inside one weight by increasing w, inside one
 * (W, w) in Landslide order.  Ranks, membership test, budget, abandonment and
 * outputs are as in orbg_decode; results depend on neither `params` nor
 * timing.
 *
 * j0: DEVICE int32 per block receiving the fitted J0, or NULL (then blocks
 * whose hard decision is already a codeword are not ranked).
 * The first call for an (n, budget rounded up to a multiple of 64) builds one
 * schedule per offset J0 = -1 .. j0max, where j0max is the largest logistic
 * weight among the first `budget` patterns taken by Hamming weight first: from
 * there on every J0 tests the same first `budget` patterns in the same order,
 * so larger fitted offsets decode with the schedule of j0max.  That takes
 * (j0max + 2) x 8 x budget bytes of device memory (about 0.2 GB for n = 127,
 * budget 10^5).  The schedules cannot hold orders whose first `budget`
 * patterns reach a logistic weight above 255 or flip more than 7 ranks above 8
 * at logistic weight 100 or more (e.g. n = 256 with a budget above 256,
 * n = 127 with a budget above about 2.86 x 10^5), nor budgets above 2^22.  Such
 * a decode (n <= 512) runs on the full m-line kernel with one segment, whose
 * fit and order are exactly the above (orbg_decode_mline with segments = 1 and
 * jdiv = 0, plus the J0 output); `params` is then unused, and the first such
 * call on a device builds the m-line decoder's table (see orbg_decode_mline).
 * Budget: 1 .. 5 x 10^6.  Errors: ORBG_EINVAL for arguments outside these
 * limits (n > 512 with an order the schedules cannot hold), as orbg_decode
 * otherwise.
 */
int orbg_decode_1line(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                      int64_t batch, uint8_t* codeword, uint64_t* queries, uint8_t* abandoned,
                      int32_t* j0, const orbg_launch_params* params, void* stream);

/*
 * Full (m-line) ORBGRAND decode (Sec. III-D; fit of Sec. III-E): per block, a piecewise-linear fit of
 * the sorted reliabilities with at most `segments` lines (anchor points from
 * ranks 1 and floor(n/2), each added anchor at the rank with the largest
 * vertical gap to the chord of its neighbouring anchors, smallest rank on
 * ties; no anchor is added when the largest gap is 0), quantized by eqs. (Q)
 * and (quant) in FP32 (round half up, capped at 2^20; a slope that is not
 * positive and finite gives the basic model); with jdiv = 1 each J_{i-1} is
 * then rounded to a multiple of beta_i (the J/beta variant).  Queries follow
 * eq. (cartP): reliability weight ascending, then the splitting patterns in the
 * nested-loop order of the integer splitting algorithm, then the Cartesian
 * product of the per-segment partial sets (segment 1 outermost; each partial
 * set by Hamming weight, then Landslide order).  Same H, llr, codeword,
 * queries, abandoned layouts and rules as orbg_decode.
 * Limits: 1 <= n <= 512, 1 <= n - k <= 64, 1 <= segments <= 4, jdiv 0 or 1,
 * 1 <= budget <= 5 x 10^6 (the threshold of Sec. IV-A; within that budget no
 * query has more than 22 flips, which bounds the device tables).  segments_out:
 * DEVICE i32 per block, the number of lines the fit used, or NULL.  The first
 * call on a device builds a 193 MB table of subset counts (allocates and
 * synchronises `stream`).  Errors: ORBG_EINVAL for arguments outside these limits, as
 * orbg_decode otherwise.
 */
int orbg_decode_mline(const uint8_t* H, const float* llr, int n, int k, uint64_t budget,
                      int64_t batch, int segments, int jdiv, uint8_t* codeword, uint64_t* queries,
                      uint8_t* abandoned, int32_t* segments_out, void* stream);

/*
 * Registers a parity-check matrix (host, as for orbg_decode) for mixed-code
 * decodes and returns its id in *code_id.  Registering the same H twice gives
 * two ids for one cached copy.  Allocates and synchronises the device on first
 * sight of an H.
 */
int orbg_code_register(const uint8_t* H, int n, int k, int* code_id);

/* Forgets a registered id (the packed columns stay cached for later use). */
int orbg_code_release(int code_id);

/*
 * Decode `batch` blocks of up to 8 different codes in one launch (basic
 * ORBGRAND as in orbg_decode, for every block with its own code).
 * codes: HOST array of `ncodes` registered ids (1 <= ncodes <= 8, every code
 * with n <= 256, the n of all codes summing to at most 2048).
 * block_code: DEVICE u8 per block, an index into `codes`; an index >= ncodes
 * decodes the block with codes[0].
 * row_offset: DEVICE i64 per block, the offset (in elements) of the block's row
 * both in `llr` (FP32, llr_len elements) and in `codeword` (bytes,
 * codeword_len elements); rows hold the block's own n values.  A row that does
 * not lie inside both buffers (offset < 0 or offset + n above either length)
 * is read as zeros and its codeword stores are dropped; its queries and flag
 * are still written.  queries/abandoned: DEVICE, one entry per block.
 * Blocks that need many queries move to the heavy pass and are searched by
 * several waves; the result is the same as orbg_decode's for each block.
 * Errors: ORBG_EINVAL for a negative length, and as orbg_decode otherwise.
 */
int orbg_decode_mixed(const int* codes, int ncodes, const uint8_t* block_code,
                      const int64_t* row_offset, const float* llr, int64_t llr_len, int64_t batch,
                      uint64_t budget, uint8_t* codeword, int64_t codeword_len, uint64_t* queries,
                      uint8_t* abandoned, const orbg_launch_params* params, void* stream);

/*
 * orbg_decode_mixed for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, layouts, rules and results, but the call allocates nothing.
 * Its work counters and heavy-block list live in a fixed array of the library
 * (about 2.1 MB per device, held until the process ends), so:
 *   - batch <= ORBG_NOALLOC_BATCH_MAX (262,144 blocks); larger batches return
 *     ORBG_EINVAL;
 *   - every code must be registered and its query schedule for this budget
 *     must exist: one orbg_decode_mixed call with the same codes and budget
 *     builds them (otherwise ORBG_EINVAL, nothing launched);
 *   - all calls on one device share that array: calls that overlap in time on
 *     one device (different streams, or host threads) race and may return wrong
 *     results; calls in one stream are ordered and safe.  The counters are
 *     cleared by a kernel at the start of every call.
 */
#define ORBG_NOALLOC_BATCH_MAX 262144
int orbg_decode_mixed_noalloc(const int* codes, int ncodes, const uint8_t* block_code,
                              const int64_t* row_offset, const float* llr, int64_t llr_len,
                              int64_t batch, uint64_t budget, uint8_t* codeword, int64_t codeword_len,
                              uint64_t* queries, uint8_t* abandoned, const orbg_launch_params* params,
                              void* stream);

/*
 * Copies the first `count` entries of the library's basic-ORBGRAND query
 * schedule for length n into the HOST buffer `out` (count x 16 bytes): entry g
 * lists the 1-based reliability ranks flipped by query g + 1 in increasing
 * order, padded with zeros (Sec. III-B/C order as described for orbg_decode).
 * 1 <= count <= 5 x 10^6 and count <= 2^n.  Synchronises `stream`.
 */
int orbg_schedule_export(int n, uint64_t count, uint8_t* out, void* stream);

/*
 * As orbg_schedule_export for the 1-line order of offset j0 (-1 <= j0 < 2^20)
 * that orbg_decode_1line uses with this `budget` (1 <= budget <= 2^22,
 * budget <= 2^n): the first `count` <= budget entries of the schedule of
 * min(j0, j0max).  *j0max (if not NULL) receives j0max.  count = 0 only builds
 * the schedules.  Errors as for orbg_decode_1line.  Synchronises `stream`.
 */
int orbg_schedule_export_1line(int n, uint64_t budget, int j0, uint64_t count, uint8_t* out,
                               int* j0max, void* stream);

/*
 * Learned batch-order proposal (an addition to the paper's method, used through
 * orbg_decode_ordered; the basic ORBGRAND order stays the fallback after the 64
 * reordered batches, and every decision is still a parity-checked codeword).
 *
 * Network: 128 -> 256 -> 256 -> 64 with ReLU; weights in BF16, accumulation in
 * FP32 on the matrix cores, activations stored in BF16, biases in FP32.
 * Parameters (caller-owned DEVICE buffers):
 *   w   FP32 [ORBG_MLP_PARAMS] masters, flat: W1 [256 x 128], b1 [256],
 *       W2 [256 x 256], b2 [256], W3 [64 x 256], b3 [64] (output x input, row-major);
 *   wb  BF16 bits [ORBG_MLP_PARAMS], the same layout rounded to nearest even;
 *   wt  BF16 bits [ORBG_MLP_TPARAMS], W1, W2, W3 transposed (input x output), in order;
 *   m, v FP32 [ORBG_MLP_PARAMS] Adam moments.
 * Calls that run the network take a DEVICE work space of at least
 * orbg_mlp_workspace_bytes(batch) bytes (1 <= batch <= 2^20); it holds the
 * activations and gradient partial sums of one call.  All calls are
 * asynchronous on `stream`.
 */
#define ORBG_MLP_PARAMS 115264
#define ORBG_MLP_TPARAMS 114688

/* Work space bytes for `batch` rows (-1 if batch is out of range). */
int64_t orbg_mlp_workspace_bytes(int64_t batch);

/* Features of `batch` blocks of length n = 128 (DEVICE llr rows): each block's
 * |LLR| values sorted ascending (the ordered reliability curve of Sec. III-A),
 * times 1/8, rounded to BF16 -> x [batch x 128] BF16 bits. */
int orbg_mlp_features(const float* llr, int n, int64_t batch, uint16_t* x, void* stream);

/* wb and wt from the FP32 masters w. */
int orbg_mlp_prepare(const float* w, uint16_t* wb, uint16_t* wt, void* stream);

/* logits [batch x 64] FP32 of features x [batch x 128]. */
int orbg_mlp_forward(const float* w, const uint16_t* wb, const uint16_t* x, int64_t batch, float* logits,
                     void* workspace, int64_t workspace_bytes, void* stream);

/* Mean softmax cross-entropy of the logits against labels (DEVICE int32 in
 * 0..63: the batch of the plain decoder's first hit) into *loss (DEVICE FP32),
 * and its gradient with respect to every parameter into grads (FP32, layout of w). */
int orbg_mlp_backward(const float* w, const uint16_t* wb, const uint16_t* wt, const uint16_t* x,
                      const int32_t* labels, int64_t batch, float* grads, float* loss, void* workspace,
                      int64_t workspace_bytes, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step counts
 * from 1) on w, m, v; refreshes wb and wt. */
int orbg_mlp_adam(float* w, float* m, float* v, const float* grads, float lr, int step, uint16_t* wb,
                  uint16_t* wt, void* stream);

/* Batch order for orbg_decode_ordered: each row of 64 logits sorted by
 * decreasing value, ties (and +0/-0) to the lower index, NaN last -> order
 * [batch x 64] u8. */
int orbg_mlp_order(const float* logits, int64_t batch, uint8_t* order, void* stream);

/* Fused inference without a work space: features (from DEVICE llr rows of
 * length 128 -- row ids[b] for output row b when ids is not NULL, else row b;
 * a row outside [0, llr_rows) gives zero features -- as orbg_mlp_features; or
 * the given BF16 features x when llr is NULL), the three layers with the
 * activations kept on chip, then logits [batch x 64] FP32 (or NULL) and/or the
 * batch order [batch x 64] u8 (or NULL) as orbg_mlp_order, with batch 0 first
 * whatever its logit when pin0 = 1.  The logits equal orbg_mlp_forward's bit
 * for bit.  0 <= batch < 2^36.  Errors: ORBG_EINVAL for a NULL input, both
 * outputs NULL or a negative llr_rows. */
int orbg_mlp_infer(const float* w, const uint16_t* wb, const float* llr, int64_t llr_rows, const int64_t* ids,
                   const uint16_t* x, int64_t batch, float* logits, uint8_t* order, int pin0, void* stream);

/*
 * Learned proposal in gated form: the network runs only for blocks the plain
 * order's first batch does not decide.
 *   1. Every block is searched over the first 64 patterns of the basic ORBGRAND
 *      order (as orbg_decode); blocks with a member there, or whose budget
 *      ends there, are written out.
 *   2. The other blocks are listed; the network (w, wb as for orbg_mlp_forward)
 *      scores their feature rows (orbg_mlp_features) and their batch order is
 *      batch 0 first (known to hold no member), then batches 1..63 by decreasing
 *      logit (ties to the lower index, NaN last).
 *   3. The listed blocks are decoded in that order as orbg_decode_ordered would
 *      (the 64 queries of batch 0 are counted, not repeated), the plain order
 *      continuing from index 4096.
 * Every block's result therefore equals orbg_decode_ordered with its own order
 * (the identity for blocks decided by batch 0), and every decision is a
 * parity-checked codeword.  H, llr, budget, codeword, queries, abandoned and
 * the errors are as for orbg_decode; n must be 128 (the network's input).
 * workspace: DEVICE, at least orbg_learned_workspace_bytes(batch) bytes.
 * order_out: DEVICE u8 [batch x 64] receiving each block's order, or NULL.
 * rest: HOST int64 receiving the number of listed blocks, or NULL.  params:
 * launch shape (NULL = defaults) of both searches; the first always stops after
 * one step, the second as orbg_decode_ex with an order.  The call
 * synchronises `stream` once, after step 1, to size the network's launches.
 */
int64_t orbg_learned_workspace_bytes(int64_t batch);
int orbg_decode_learned(const uint8_t* H, const float* llr, int n, int k, uint64_t budget, int64_t batch,
                        const float* w, const uint16_t* wb, void* workspace, int64_t workspace_bytes,
                        uint8_t* codeword, uint64_t* queries, uint8_t* abandoned, uint8_t* order_out,
                        int64_t* rest, const orbg_launch_params* params, void* stream);

/* Message describing the calling thread's last non-OK status ("" if none). */
const char* orbg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ORBGRAND_H */
