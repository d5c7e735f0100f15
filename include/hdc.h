/*
 * hdc.h -- C ABI of libhdc.so, the MI355X (gfx950) HDC classification hot
 * path: random-projection encoding with binarisation, majority bundling,
 * Hamming distance under reduction perforation, argmin, the fused
 * classifier and a one-launch evaluation of many approximation
 * configurations (arXiv 2606.26547).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is DEVICE memory owned by the caller,
 *   except where a comment says "host".  The library allocates no device
 *   memory in any call; scratch comes from the caller's `ws` buffer, sized
 *   by the matching *_workspace_bytes() function.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream).  Every call only enqueues work on that stream and returns;
 *   outputs are valid once the stream has reached that point.  Calls on one
 *   stream are ordered; calls sharing a workspace must not overlap.
 * Errors.  Arguments are validated synchronously before anything is
 *   enqueued: HDC_ERR_INVALID for a NULL required pointer, a negative count,
 *   non-positive F / D / K, a leading dimension that is too small or
 *   misaligned, or an empty/out-of-range dimension set; HDC_ERR_UNSUPPORTED
 *   for a feature-type / compute-type pair or a size outside the compiled
 *   kernels; HDC_ERR_WORKSPACE when ws_bytes is below the required size;
 *   HDC_ERR_DEVICE when a launch fails.  n == 0 enqueues nothing and returns
 *   HDC_OK.  No exception crosses the ABI.
 * Hypervectors.  A binary hypervector is a row of uint64 words; bit j of
 *   word w is element 64*w + j (LSB first, little-endian words).  A set bit
 *   encodes the bipolar value -1, a clear bit +1.  Bits past the last
 *   element of a row are written as 0 and must be 0 on input.
 * Dimension sets.  hdc_dims {start, end, stride} selects the dimensions
 *   S = { start + j*stride : start + j*stride < end } of a D-dimensional
 *   hypervector, in that order; {0, D, 1} is "no approximation".  This is
 *   the paper's reduction perforation (start offset, end offset, stride;
 *   Sec. 2.2 Listing 1 and Sec. 4.2 "Reduction Perforation"); truncating
 *   the encoding dimensionality to D' (Sec. 4.2 "Encoding Dimensionality")
 *   is {0, D', 1}.  Requires 0 <= start < end <= D and stride >= 1.
 * Features.  X is row-major [n][ldx] of `x_type` elements.  Only columns
 *   [0, F) are read as features; ldx must be >= F rounded up to 64 and a
 *   multiple of 16 elements, and X 16-byte aligned (the pad columns are
 *   read but ignored).
 * Projection.  P is the random +-1 projection hypermatrix stored
 *   row-major [D][ldp] int8 (row d holds the F weights of dimension d, i.e.
 *   P = B^T for the paper's random-projection matrix B; Sec. 2.2 Listing
 *   1's hypermatrix<D, F>).  ldp >= F rounded up to 64, a multiple of 16,
 *   P 16-byte aligned; columns [0, F) must hold +1 or -1.  D * ldp must be
 *   below 2^32 bytes (the kernels address P with 32-bit offsets); a larger
 *   projection gives HDC_ERR_UNSUPPORTED.  With compute HDC_INT8_SHIFTED,
 *   P is the shifted form written by hdc_shift_projection instead (columns
 *   [0, F) hold p + 1, i.e. 0 or 2); the results are those of HDC_INT8 on
 *   the +-1 projection it was made from.  Likewise HDC_FP8_E4M3_SHIFTED
 *   reads the E4M3 form (bytes 0x00 / 0x40) and gives the results of
 *   HDC_FP8_E4M3.
 */
#ifndef HDC_H
#define HDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HDC_OK = 0,
    HDC_ERR_INVALID = 1,
    HDC_ERR_UNSUPPORTED = 2,
    HDC_ERR_WORKSPACE = 3,
    HDC_ERR_DEVICE = 4
} hdc_status;

/* Feature types (x_type) and encoding compute types (compute).
 * Supported (x_type -> compute) pairs:
 *   HDC_INT8 / HDC_UINT8 -> HDC_INT8     exact: int8 MFMA, int32 accumulation
 *                                        (uint8 runs as x-128 plus a column-sum
 *                                        correction, also exact)
 *   HDC_INT8 / HDC_UINT8 -> HDC_BF16     bf16 MFMA, fp32 accumulation
 *   HDC_INT8 / HDC_UINT8 -> HDC_FP8_E4M3 OCP E4M3 MFMA, fp32 accumulation
 *   HDC_INT8 / HDC_UINT8 -> HDC_FP8_E4M3_SPLIT
 *                                        each feature x written as
 *                                        16*floor(x/16) + (x mod 16), both
 *                                        parts exact in E4M3; two E4M3 MFMAs
 *                                        into fp32 sums below 2^24: exact,
 *                                        the same bits as HDC_INT8
 *   HDC_INT8 -> HDC_INT8_SHIFTED          exact, the same bits as HDC_INT8, on
 *                                        the shifted projection (see
 *                                        hdc_shift_projection): int8 MFMA on
 *                                        weights p + 1 in {0, 2}, every sum
 *                                        started from minus the query's
 *                                        feature sum
 *   HDC_INT8 / HDC_UINT8 -> HDC_FP8_E4M3_SHIFTED
 *                                        the same bits as HDC_FP8_E4M3, on
 *                                        the shifted projection in E4M3
 *                                        bytes (0 / 2.0): E4M3 MFMA, every
 *                                        sum started from minus the sum of
 *                                        the query's rounded features
 *   HDC_FP32 -> HDC_FP32 / HDC_BF16 / HDC_FP8_E4M3   (F <= 256)
 * The reduced types round each feature to the compute type (round to nearest
 * even) and multiply by the exactly representable +-1 weights (Sec. 4.2
 * "Element Type Representation").  HDC_FP8_E4M3_SPLIT is a compute type
 * only (never a feature type) and is not a sweep configuration dtype; so
 * are HDC_INT8_SHIFTED and HDC_FP8_E4M3_SHIFTED. */
typedef enum {
    HDC_INT8 = 0,
    HDC_UINT8 = 1,
    HDC_BF16 = 2,
    HDC_FP8_E4M3 = 3,
    HDC_FP32 = 4,
    HDC_FP8_E4M3_SPLIT = 5,
    HDC_INT8_SHIFTED = 6,
    HDC_FP8_E4M3_SHIFTED = 7
} hdc_dtype;

typedef struct {
    int32_t start, end, stride;
} hdc_dims;

/* Human-readable name of a status code (static string). */
const char *hdc_status_string(hdc_status s);

/* Number of dimensions in a dimension set (0 when it is empty/invalid). */
int32_t hdc_dims_count(hdc_dims dims);

/* ---------------------------------------------------------------------
 * hdc_encode -- random-projection encoding followed by binarisation
 * (Sec. 2.2 Listing 1, the matmul primitive; Sec. 4.2 "Automatic
 * Binarization").  For each query row i and the j-th dimension d = S_j:
 *     y = sum_{f<F} x'[i][f] * P[d][f],   bit j of H row i = (y < 0)
 * where x' is the feature under `compute`; y == 0 gives +1 (bit 0).  Only
 * the |S| selected dimensions are computed; they are packed densely, so a
 * row holds ceil(|S|/64) words.
 *   H   [n][ldh] uint64, ldh >= ceil(|S|/64); words past that are untouched.
 * A batch too small to fill the device spreads the dimensions over several
 * workgroups per query block (each writes whole words of its own).
 * ------------------------------------------------------------------- */
hdc_status hdc_encode(void *stream,
                      const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                      const int8_t *P, int32_t D, int64_t ldp,
                      hdc_dtype compute, hdc_dims dims,
                      uint64_t *H, int64_t ldh);
/* hdc_encode with the kernel shape named (a tile variant of the encode
 * bucket, see hdc_tile_variants; 0 = the built-in rule, as hdc_encode);
 * a variant the bucket is not compiled with gives HDC_ERR_UNSUPPORTED. */
hdc_status hdc_encode_tiled(void *stream,
                            const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                            const int8_t *P, int32_t D, int64_t ldp,
                            hdc_dtype compute, hdc_dims dims,
                            uint64_t *H, int64_t ldh, int32_t tile);

/* ---------------------------------------------------------------------
 * hdc_shift_projection -- the projection in the form a shifted compute
 * type reads: out[d][f] = P[d][f] + 1 for f < F (0 or 2 for +-1 weights),
 * as int8 (compute = HDC_INT8_SHIFTED) or as E4M3 bytes 0x00 / 0x40
 * (compute = HDC_FP8_E4M3_SHIFTED), and 0 in the pad columns [F, ldo).  The
 * encoding is unchanged (Sec. 2.2 Listing 1; with x the features and p a
 * row, sum_f x_f (p_f + 1) - sum_f x_f is the same y); the shifted weights
 * are mostly zero bits, which the matrix cores run at a higher clock than
 * +-1.  Made once per model.  Another compute gives HDC_ERR_UNSUPPORTED.
 *   P    [D][ldp] int8, as for hdc_encode (+-1 in columns [0, F))
 *   out  [D][ldo] int8 output, ldo >= F rounded up to 64, a multiple of
 *        16, 16-byte aligned; D * ldo below 2^32 bytes.  out may be P
 *        itself when ldo == ldp (in place); any other overlap with P gives
 *        HDC_ERR_INVALID.
 * F <= 1024.
 * ------------------------------------------------------------------- */
hdc_status hdc_shift_projection(void *stream,
                                const int8_t *P, int32_t D, int32_t F, int64_t ldp,
                                hdc_dtype compute, int8_t *out, int64_t ldo);

/* ---------------------------------------------------------------------
 * hdc_bundle -- class bundling (Sec. 2.1: same-class hypervectors are
 * aggregated into one class hypervector), as the per-dimension majority:
 *     n_k = #{i : labels[i] == k},  cnt[k][d] = #{i in class k : bit d set}
 *     C bit d of class k = (2 * cnt[k][d] > n_k)
 * so a tie gives +1 and an empty class is all +1.  Exact and deterministic
 * (integer counts; the order rows are visited does not matter).
 *   H       [n][ldh] uint64 hypervectors of nbits elements each, 8-byte
 *           aligned
 *   labels  [n] int32 in [0, K) (precondition; out-of-range rows are skipped)
 *   C       [K][ldc] uint64 output, ldc >= ceil(nbits/64): words 0 ..
 *           ceil(nbits/64) - 1 of every class row are written (bits past
 *           nbits 0), words past them are left as they are
 *   counts  [K] int32 output n_k (every entry written), may be NULL
 *   ws      >= hdc_bundle_workspace_bytes(n, nbits, K) bytes, 256-byte
 *           aligned (the class sums, a row index list grouped by class and
 *           its offsets)
 * Supports K <= 128 and n < 2^30.
 * ------------------------------------------------------------------- */
size_t hdc_bundle_workspace_bytes(int64_t n, int32_t nbits, int32_t K);
hdc_status hdc_bundle(void *stream,
                      const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                      const int32_t *labels, int32_t K,
                      uint64_t *C, int64_t ldc, int32_t *counts,
                      void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------
 * hdc_bundle_noalloc -- hdc_bundle for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments without the workspace, the same
 * results bit for bit.  Scratch is a fixed array inside the library, one
 * copy per device (held until the process ends; its address is looked up
 * on the first call on a device, with that device current), of
 * hdc_bundle_noalloc_limit_bytes() bytes (32 MiB): a call whose
 * hdc_bundle_workspace_bytes(n, nbits, K) exceeds that returns
 * HDC_ERR_UNSUPPORTED before any device work.  The call allocates nothing
 * and clears what must start at zero itself.  Every call on a device
 * shares that device's array: calls that may overlap on one device (other
 * streams, other host threads) race and must be serialised by the caller.
 * The work runs on the device current at the call.
 * ------------------------------------------------------------------- */
size_t hdc_bundle_noalloc_limit_bytes(void);
hdc_status hdc_bundle_noalloc(void *stream,
                              const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                              const int32_t *labels, int32_t K,
                              uint64_t *C, int64_t ldc, int32_t *counts);

/* ---------------------------------------------------------------------
 * hdc_class_acc / hdc_retrain_epoch -- retraining (Sec. 5: the apps'
 * TRAIN_ITERATIONS knob, whose iterations the tuner cuts; the update rule
 * itself is not stated in the paper, the one implemented is the usual
 * perceptron-style rule applied to a whole epoch).  With b_i the bipolar
 * form of row i of H (+1 for bit 0, -1 for bit 1):
 *   hdc_class_acc:     acc[k][d] = sum over rows i with labels[i] == k of
 *                      b_i(d)  (the sum that majority bundling thresholds)
 *   hdc_retrain_epoch: for every row with pred[i] != labels[i],
 *                      acc[labels[i]] += b_i and acc[pred[i]] -= b_i
 * Both then write the model C: bit d of class k is 1 exactly when
 * acc[k][d] < 0 (zero gives +1, the bundling tie rule).  pred is the label
 * each row gets from the model at the start of the epoch (e.g. from
 * hdc_hamming_argmin over all nbits).  Integer updates: the result does not
 * depend on the order rows are visited.
 *   H       [n][ldh] uint64 training hypervectors (nbits valid bits),
 *           8-byte aligned
 *   labels  [n] int32 in [0, K)   pred [n] int32 in [0, K) (rows with a
 *           label or prediction outside [0, K) are skipped)
 *   acc     [K][nbits] int32, written (class_acc) / updated (epoch)
 *   C       [K][ldc] uint64 output, ldc >= ceil(nbits / 64)
 *   n_wrong device int32 output (rows with pred != label), may be NULL
 *   ws      >= hdc_retrain_workspace_bytes(n, nbits, K) bytes, 256-byte
 *           aligned (one size serves both calls)
 * Supports K <= 128 and n < 2^30.
 * ------------------------------------------------------------------- */
size_t hdc_retrain_workspace_bytes(int64_t n, int32_t nbits, int32_t K);
hdc_status hdc_class_acc(void *stream,
                         const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                         const int32_t *labels, int32_t K,
                         int32_t *acc, uint64_t *C, int64_t ldc,
                         void *ws, size_t ws_bytes);
hdc_status hdc_retrain_epoch(void *stream,
                             const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                             const int32_t *labels, const int32_t *pred, int32_t K,
                             int32_t *acc, uint64_t *C, int64_t ldc, int32_t *n_wrong,
                             void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------
 * hdc_hamming_argmin -- Hamming distance of each query hypervector to every
 * class hypervector with reduction perforation, then argmin (Sec. 2.2
 * Listing 1: hamming_distance, red_perf, arg_min; Sec. 4.2).
 *     dist[i][k] = #{ d in S(perf) : bit d of Q row i != bit d of C row k }
 * The count is used as-is (not rescaled).  argmin[i] is the lowest k with
 * the smallest distance.
 *   nbits    valid bits of each Q and C row (hypervector length); requires
 *            perf.end <= nbits, ldq and ldc >= ceil(nbits / 64)
 *   Q        [n][ldq] uint64,  C [K][ldc] uint64
 *   argmin   [n] int32 output
 *   min_dist [n] int32 output, may be NULL
 *   dists    [n][K] int32 output, may be NULL
 * Supports K <= 128.
 * ------------------------------------------------------------------- */
hdc_status hdc_hamming_argmin(void *stream,
                              const uint64_t *Q, int64_t n, int64_t ldq,
                              const uint64_t *C, int32_t K, int64_t ldc,
                              int32_t nbits, hdc_dims perf,
                              int32_t *argmin, int32_t *min_dist, int32_t *dists);

/* ---------------------------------------------------------------------
 * hdc_hamming_prepare / hdc_hamming_argmin_prepared -- the same search as
 * hdc_hamming_argmin, split in two for resident class hypervectors (Sec. 2.2
 * Listing 1: hamming_distance, red_perf, arg_min; Sec. 4.2): _prepare turns
 * the classes and the perforation set S(perf) into a matrix-core operand
 * in the workspace once; _prepared then searches any number of query
 * batches against it.  Outputs are identical to hdc_hamming_argmin with the
 * same arguments.  `ws` must stay untouched between the calls; K and perf
 * must be the same in both.
 *   Q        16-byte aligned with an even row pitch ldq <= 2^20 (the
 *            prepared search streams query words 16 bytes at a time)
 *   ws       >= hdc_hamming_workspace_bytes(perf, K) bytes, 16-byte aligned
 * Supports K <= 128, perf.end <= 65536.
 * ------------------------------------------------------------------- */
size_t hdc_hamming_workspace_bytes(hdc_dims perf, int32_t K);
hdc_status hdc_hamming_prepare(void *stream,
                               const uint64_t *C, int32_t K, int64_t ldc,
                               hdc_dims perf, void *ws, size_t ws_bytes);
hdc_status hdc_hamming_argmin_prepared(void *stream,
                                       const uint64_t *Q, int64_t n, int64_t ldq,
                                       int32_t K, hdc_dims perf,
                                       int32_t *argmin, int32_t *min_dist, int32_t *dists,
                                       const void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------
 * hdc_cosine_prepare / hdc_cosine_argmax_prepared -- cosine similarity of
 * binary query hypervectors against NON-binarised class hypervectors, the
 * alternative to Hamming distance the paper weighs in Sec. 3 "Algorithmic
 * Choice" (integer class accumulators kept as they are, similarity by
 * normalised dot product), under reduction perforation (Sec. 4.2).  With b
 * the bipolar form of the query (+1 for bit 0, -1 for bit 1) and a_k the
 * class accumulator (e.g. hdc_class_acc / hdc_retrain_epoch output):
 *     score[i][k] = (double)(sum over d in S of b(d) * a_k(d))
 *                   * (1 / sqrt(sum over d in S of a_k(d)^2))
 * with the dot product exact (integer), the reciprocal square root and the
 * product each correctly rounded in double, and 0 as the factor of an
 * all-zero class over S.  The query's own norm is the same for every class
 * and does not change the ranking; it is left out.  label[i] is the lowest
 * k with the largest score.  _prepare builds the matrix-core operand, the
 * per-class sums and norms in the workspace once; _argmax_prepared
 * searches any number of query batches against it.  `ws` must stay
 * untouched between the calls; K and perf must be the same in both.
 *   acc      [K][lda] int32, lda >= perf.end; every entry over S must lie
 *            in [-32639, 32639]: otherwise _prepare marks the workspace
 *            and every label the search writes is -1 and every score NaN
 *   Q        [n][ldq] uint64 (>= perf.end valid bits), 16-byte aligned,
 *            even ldq <= 2^20
 *   label    [n] int32 output; max_score [n], scores [n][K] double, may be
 *            NULL
 *   ws       >= hdc_cosine_workspace_bytes(perf, K) bytes, 16-byte aligned
 * Supports K <= 128, perf.end <= 65536.
 * ------------------------------------------------------------------- */
size_t hdc_cosine_workspace_bytes(hdc_dims perf, int32_t K);
hdc_status hdc_cosine_prepare(void *stream,
                              const int32_t *acc, int32_t K, int64_t lda,
                              hdc_dims perf, void *ws, size_t ws_bytes);
hdc_status hdc_cosine_argmax_prepared(void *stream,
                                      const uint64_t *Q, int64_t n, int64_t ldq,
                                      int32_t K, hdc_dims perf,
                                      int32_t *label, double *max_score, double *scores,
                                      const void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------
 * hdc_adc_argmax -- dot-product similarity as an in-memory accelerator
 * computes it (Sec. 3 "In-Memory Accelerator Approximations": (I) ADC
 * resolution, (III) analog quantization scale; Sec. 6 SpecPCM: dot
 * products over 128-element array chunks, each partial product quantized
 * by the ADC before accumulation).  For query i and class k, with b the
 * bipolar form of a hypervector (+1 for bit 0, -1 for bit 1) and chunk c
 * the dimensions [128c, 128c+128) that lie in S(perf):
 *     s_c   = sum over d in chunk c of b_q(d) * b_k(d)
 *     x     = min(max(s_c, adc.floor), adc.ceil)
 *     code  = min(floor((x - adc.floor) / adc.step + 1/2), 2^adc.res_bits - 1)
 *     score = sum over chunks holding a dimension of S of adc.floor + adc.step * code
 * label[i] is the lowest k with the largest score.  The paper's reference
 * configuration {8, 1, -127, 128} reproduces the unquantized dot product
 * (except a partial of -128, which clips to -127).
 *   Q [n][ldq], C [K][ldc] uint64 (>= perf.end valid bits)
 *   label [n] int32 output; max_score [n], scores [n][K] int32, may be NULL
 * Supports K <= 128, perf.end <= 65536, 1 <= res_bits <= 16, step >= 1,
 * floor <= ceil.
 * ------------------------------------------------------------------- */
typedef struct {
    int32_t res_bits, step, floor, ceil;
} hdc_adc;

hdc_status hdc_adc_argmax(void *stream,
                          const uint64_t *Q, int64_t n, int64_t ldq,
                          const uint64_t *C, int32_t K, int64_t ldc,
                          hdc_dims perf, hdc_adc adc,
                          int32_t *label, int32_t *max_score, int32_t *scores);

/* ---------------------------------------------------------------------
 * hdc_adc_prepare / hdc_adc_argmax_prepared -- the similarity of
 * hdc_adc_argmax (same definition, same outputs bit for bit) split in two
 * for resident class hypervectors: _prepare turns the classes and the
 * perforation set S(perf) into a matrix-core operand and per-chunk counts
 * in the workspace once; _argmax_prepared searches any number of query
 * batches under any ADC setting against it.  `ws` must stay untouched
 * between the calls; K and perf must be the same in both.
 *   Q        [n][ldq] uint64 (>= perf.end valid bits), 16-byte aligned,
 *            even ldq <= 2^20
 *   ws       >= hdc_adc_workspace_bytes(perf, K) bytes, 16-byte aligned
 * Supports K <= 128, perf.end <= 65536, and the ADC settings of
 * hdc_adc_argmax.
 * ------------------------------------------------------------------- */
size_t hdc_adc_workspace_bytes(hdc_dims perf, int32_t K);
hdc_status hdc_adc_prepare(void *stream,
                           const uint64_t *C, int32_t K, int64_t ldc,
                           hdc_dims perf, void *ws, size_t ws_bytes);
hdc_status hdc_adc_argmax_prepared(void *stream,
                                   const uint64_t *Q, int64_t n, int64_t ldq,
                                   int32_t K, hdc_dims perf, hdc_adc adc,
                                   int32_t *label, int32_t *max_score, int32_t *scores,
                                   const void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------
 * hdc_classify -- the fused inference path of Sec. 2.2 Listing 1 (matmul,
 * then hamming_distance under red_perf, then arg_min) in one kernel, with
 * the binarisation of Sec. 4.2 "Automatic Binarization" between them:
 * encode each query over the dimensions S(dims) under `compute`, compare
 * bit j of the query with bit S_j of each (full-D) class hypervector,
 * argmin.  Equal, bit for bit, to
 * hdc_encode(dims) followed by hdc_hamming_argmin over the gathered class
 * bits, without writing the query hypervectors anywhere.
 *   C       [K][ldc] uint64 class hypervectors over all D dimensions
 *           (as written by hdc_bundle with nbits = D)
 *   labels  [n] int32 output;  dists [n][K] int32 output, may be NULL
 *   ws      >= hdc_classify_workspace_bytes(hdc_dims_count(dims), K)
 *   scratch optional (may be NULL), 4-byte aligned: with
 *           hdc_classify_scratch_bytes(n, hdc_dims_count(dims), K) bytes a
 *           batch too small to fill the device spreads its dimensions over
 *           several workgroups per query block, which add their integer
 *           partial sums there before a small argmin kernel (a smaller
 *           scratch allows fewer splits; NULL or 0 bytes, none).  The
 *           results are the same either way.  Calls sharing a scratch
 *           must not overlap.
 *   tile    the kernel shape: a tile variant of the classify bucket (see
 *           hdc_tile_variants) or 0 for the built-in rule; a variant the
 *           bucket is not compiled with gives HDC_ERR_UNSUPPORTED
 * Supports K <= 128, F <= 1024.
 * ------------------------------------------------------------------- */
size_t hdc_classify_workspace_bytes(int32_t n_dims, int32_t K);
size_t hdc_classify_scratch_bytes(int64_t n, int32_t n_dims, int32_t K);
hdc_status hdc_classify(void *stream,
                        const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                        const int8_t *P, int32_t D, int64_t ldp,
                        hdc_dtype compute, hdc_dims dims,
                        const uint64_t *C, int32_t K, int64_t ldc,
                        int32_t *labels, int32_t *dists,
                        void *ws, size_t ws_bytes, void *scratch, size_t scratch_bytes, int32_t tile);

/* ---------------------------------------------------------------------
 * hdc_classify_prepare / hdc_classify_prepared -- hdc_classify split in
 * two, for resident models (Sec. 2.2 Listing 1; Sec. 4.2): _prepare
 * gathers the class hypervectors over S(dims) into the workspace once (the
 * class operand of the fused kernel and the per-class count of -1
 * elements); _prepared then classifies any number of query batches with
 * that workspace, launching only the fused kernel (plus the argmin kernel
 * of a dimension-split launch, see `scratch` above).  The result is
 * identical to hdc_classify.  `ws` must stay untouched between the two
 * calls and be sized by hdc_classify_workspace_bytes(); K and dims must be
 * the same in both calls.
 * ------------------------------------------------------------------- */
hdc_status hdc_classify_prepare(void *stream,
                                const uint64_t *C, int32_t K, int64_t ldc, hdc_dims dims,
                                void *ws, size_t ws_bytes);
hdc_status hdc_classify_prepared(void *stream,
                                 const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                                 const int8_t *P, int32_t D, int64_t ldp,
                                 hdc_dtype compute, hdc_dims dims, int32_t K,
                                 int32_t *labels, int32_t *dists,
                                 const void *ws, size_t ws_bytes, void *scratch, size_t scratch_bytes,
                                 int32_t tile);

/* ---------------------------------------------------------------------
 * hdc_eval_configs -- one call that evaluates many approximation
 * configurations on the same queries (a persistent kernel over per-
 * configuration work items, and/or the shared path; see the sweep tile
 * variants below): the inner loop of the paper's tuning system, which runs
 * each candidate configuration and reads back its quality of service and
 * time (Sec. 3, Sec. 4.1).  For every
 * configuration c, the queries are classified exactly as hdc_classify with
 * dims {cfg.start, cfg.d_trunc, cfg.stride} and compute = cfg.dtype, and
 *     out[c].correct   = #{i : label_i == truth[i]}
 *     out[c].n         = n (0 for a configuration that does no work)
 *     out[c].device_us = device wall-clock time summed over c's work items
 * (several items run concurrently, so this is busy time, not elapsed time;
 * for a configuration on the shared path, the time of the search items
 * that rank it, which it shares with the other configurations of its
 * chain, without the shared encoding).
 * A configuration with an unsupported dtype or an empty / out-of-range
 * dimension set does no work and reports n = 0.  Work is scheduled longest
 * configuration first.
 *   X      integer features only (HDC_INT8 / HDC_UINT8); F <= 1024
 *   truth  [n] int32 true labels (device)
 *   cfgs   [ncfg] hdc_config, HOST memory, read before the call returns;
 *          ncfg <= 4096.  tile_id: the work-item shape of that
 *          configuration, a sweep variant of the (x_type, F, K) bucket
 *          (HDC_TILE_SWEEP_*; see hdc_tile_variants) or 0 for the built-in
 *          one (items of 256 queries); a variant the bucket is not compiled
 *          with, or a negative id, gives HDC_ERR_UNSUPPORTED before any
 *          device work
 *   out    [ncfg] hdc_config_result, HOST memory, overwritten; valid once
 *          the stream has passed the call (into page-locked memory the copy
 *          is asynchronous; into pageable memory the call returns only
 *          after the results have arrived)
 *   ws     >= hdc_eval_configs_workspace_bytes(ncfg, F, D, K), 256-byte
 *          aligned (per-configuration class operands, the projection rows
 *          converted to E4M3 for the direct-staged body, and the shared
 *          path's two encodings of 4096 queries at a time)
 *   max_workgroups  0: as many workgroups as fit on the device at once;
 *          otherwise at most this many (a configuration job that shares
 *          the device with latency-bound inference leaves it room; the
 *          work queue finishes every item whatever the count).  It bounds
 *          the persistent kernel only, not the shared path's launches
 * ------------------------------------------------------------------- */
typedef struct {
    int32_t d_trunc, stride, start;
    int32_t dtype;          /* hdc_dtype compute type */
    int32_t tile_id;        /* HDC_TILE_SWEEP_* or 0 */
} hdc_config;

typedef struct {
    int32_t correct;
    int32_t n;
    double device_us;
} hdc_config_result;

size_t hdc_eval_configs_workspace_bytes(int32_t ncfg, int32_t F, int32_t D, int32_t K);
hdc_status hdc_eval_configs(void *stream,
                            const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                            const int32_t *truth,
                            const int8_t *P, int32_t D, int64_t ldp,
                            const uint64_t *C, int32_t K, int64_t ldc,
                            const hdc_config *cfgs, int32_t ncfg,
                            hdc_config_result *out,
                            void *ws, size_t ws_bytes, int32_t max_workgroups);

/* ---------------------------------------------------------------------
 * Tile variants -- the kernel shapes each launch can take, for an autotuner
 * that times the variants of a shape on the device and then names the
 * fastest in each call (hdc_encode_tiled, hdc_classify(_prepared), the
 * tile_id of each hdc_eval_configs configuration).  The library holds no
 * mutable tile state.  A bucket is (kind, x_type, compute, the compiled
 * feature width the launch uses for F, the class tiles of K: 1, 2 or 4 for
 * K <= 32, 64, 128; the sweep compiles 1 or 4).  Every variant of a bucket
 * computes identical results; only the time differs.
 *   kind      HDC_KERNEL_ENCODE (hdc_encode_tiled), HDC_KERNEL_CLASSIFY
 *             (hdc_classify, hdc_classify_prepared), HDC_KERNEL_SWEEP
 *             (hdc_eval_configs; compute is ignored, x_type is the
 *             feature type of the job)
 *   variants  encoder / classifier: HDC_TILE_DMA_2X2 and HDC_TILE_DMA_1X1
 *             (projection staged straight into LDS; two query tiles x two
 *             dimension tiles per wave, or one of each; int8 features on the
 *             int8 path), HDC_TILE_DMA_2X3 (classifier only, one class tile,
 *             F <= 640: two query tiles x three dimension tiles, 96-
 *             dimension chunks in two LDS stages; it cannot split its
 *             dimensions, so a batch too small to fill the device runs on
 *             the 2x2 shape with dimension splits instead),
 *             HDC_TILE_REG_QT2 and HDC_TILE_REG_QT1 (register
 *             staging, two or one query tiles of 32 per wave);
 *             sweep: HDC_TILE_SWEEP_256 (work items of 256 queries: int8
 *             configurations take two query tiles per wave where the
 *             registers allow), HDC_TILE_SWEEP_128 (items of 128) and
 *             HDC_TILE_SWEEP_256_DMA (items of 256 on direct-staged bodies:
 *             int8 configurations on the classifier's HDC_TILE_DMA_2X2
 *             body with int8 features, E4M3 configurations on the same 2x2
 *             shape reading projection rows converted once per launch,
 *             bf16 configurations as HDC_TILE_SWEEP_256; K <= 32,
 *             F <= 640) and HDC_TILE_SWEEP_SHARED (every bucket: the
 *             configurations with this tile take their distances from one
 *             encoding of the union of their dimension sets per encoding
 *             -- int8, which bf16 configurations share since integer
 *             features make the two identical, and E4M3 -- by masked
 *             Hamming distance; a configuration's set depends only on its
 *             own start, stride and end, and the set of configurations
 *             with one start and stride is searched in one pass whose
 *             prefix sums give every end; same counts, no per-configuration
 *             encode)
 * hdc_tile_variants writes up to `cap` (host array) variant ids the bucket
 * is compiled with, the built-in choice first, and returns how many there
 * are, or -1 for a shape outside the compiled kernels.
 * ------------------------------------------------------------------- */
typedef enum {
    HDC_KERNEL_ENCODE = 0,
    HDC_KERNEL_CLASSIFY = 1,
    HDC_KERNEL_SWEEP = 2
} hdc_kernel;

enum {
    HDC_TILE_DMA_2X2 = 1,
    HDC_TILE_DMA_1X1 = 2,
    HDC_TILE_REG_QT1 = 3,
    HDC_TILE_REG_QT2 = 4,
    HDC_TILE_DMA_2X3 = 5,
    HDC_TILE_SWEEP_128 = 1,
    HDC_TILE_SWEEP_256 = 2,
    HDC_TILE_SWEEP_256_DMA = 3,
    HDC_TILE_SWEEP_SHARED = 4
};

int32_t hdc_tile_variants(hdc_kernel kind, hdc_dtype x_type, hdc_dtype compute, int32_t F, int32_t K,
                          int32_t *variants, int32_t cap);

/* Frequency in Hz of the device wall clock (the one hdc_eval_configs times
 * work items with). */
double hdc_device_clock_hz(void);

/* ---------------------------------------------------------------------
 * hdc_feature_perforate -- reduction perforation applied to the encoding's
 * own reduction, the one over features (Sec. 4.2 "Reduction Perforation":
 * a perforated matrix-vector product is rescaled for the iterations it
 * skips).  Copies the columns S(fperf) = { fperf.start + j*fperf.stride <
 * fperf.end } of a row-major matrix into a dense one, so that hdc_encode /
 * hdc_classify on the result with F' = |S(fperf)| features compute the
 * perforated product.  The rescale factor F/F' is positive and changes no
 * sign, so the binarised encoding needs no rescale.  Apply it to the
 * features X and, once per configuration, to the projection rows P (int8,
 * n = D).
 *   X   [n][ldx] of x_type (HDC_INT8, HDC_UINT8 or HDC_FP32), ldx >= F
 *   Y   [n][ldy]: column j < F' holds X column fperf.start + j*fperf.stride,
 *       columns F'..ldy-1 are 0; ldy >= F', ldy * element size a multiple
 *       of 16 bytes, Y 16-byte aligned
 * Requires 0 <= fperf.start < fperf.end <= F, fperf.stride >= 1.
 * ------------------------------------------------------------------- */
hdc_status hdc_feature_perforate(void *stream,
                                 const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                                 hdc_dims fperf, void *Y, int64_t ldy);

/* ---------------------------------------------------------------------
 * hdc_level_quantize / hdc_level_id_encode -- Level-ID encoding, the
 * ID-based alternative to random projection (Sec. 3 "Algorithmic Choice";
 * Sec. 5.3: the Level knob, how many discrete levels continuous features
 * are quantised to before they map to hypervectors).
 * _quantize: for feature f of row i, in binary32 with every operation
 * rounded to nearest even and nothing fused,
 *     v = ((x - lo[f]) * L) / (hi[f] - lo[f])
 *     lev[i][f] = 0 if hi[f] - lo[f] is not > 0 or v is not > 0 (NaN
 *                 included), L - 1 if v >= L - 1, floor(v) otherwise.
 *   X [n][ldx] float, lo / hi [F] float, lev [n][ldl] uint16 output,
 *   ldx, ldl >= F; 1 <= L <= 65535.
 * _encode: with b(row, d) = +1 for bit 0 and -1 for bit 1,
 *     s = sum over f < F of b(ID_f, d) * b(LV_lev[i][f], d)
 *     bit d of H row i = (s < 0)   (s == 0 gives +1)
 * i.e. the bundle of the bound (ID, level) pairs of the row.  The identity
 * hypervectors ID [F][ldid] and level hypervectors LV [L][ldlv] are inputs
 * (packed, D bits, pad bits 0); lev entries must be < L (a larger entry
 * reads as L - 1).  H [n][ldh] uint64 output, pad bits written as 0.
 *   ldid, ldlv, ldh >= ceil(D / 64); for _encode, lev 16-byte aligned
 *   and ldl >= F rounded up to a multiple of 8 (levels are read 8 at a
 *   time; the pad entries are read and ignored).
 * Supports F <= 1024, L <= 1024.
 * ------------------------------------------------------------------- */
hdc_status hdc_level_quantize(void *stream,
                              const float *X, int64_t n, int32_t F, int64_t ldx,
                              const float *lo, const float *hi, int32_t L,
                              uint16_t *lev, int64_t ldl);
hdc_status hdc_level_id_encode(void *stream,
                               const uint16_t *lev, int64_t n, int32_t F, int64_t ldl,
                               const uint64_t *ID, int64_t ldid,
                               const uint64_t *LV, int32_t L, int64_t ldlv,
                               int32_t D, uint64_t *H, int64_t ldh);

/* ---------------------------------------------------------------------
 * hdc_convert_features -- diagnostic: the value each feature takes inside
 * the encoder under `compute` (the device conversion the kernels use),
 * written as float: out[i][f] for f < F.  out is [n][F] float.
 * ------------------------------------------------------------------- */
hdc_status hdc_convert_features(void *stream,
                                const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                                hdc_dtype compute, float *out);

#ifdef __cplusplus
}
#endif
#endif
