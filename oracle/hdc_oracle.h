/*
 * hdc_oracle.h -- plain CPU oracle for the HDC classification hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference that
 * the GPU path is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header, table or constant with the GPU library.
 *
 * Everything here is a direct, slow transcription of the operations the
 * paper defines (arXiv 2606.26547):
 *   - random-projection encoding, a hypervector-times-hypermatrix product
 *     followed by binarisation to {+1,-1} stored one bit per element
 *     (Sec. 2.2 Listing 1; Sec. 4.2 "Automatic Binarization");
 *   - class bundling, aggregation of the hypervectors of each class
 *     (Sec. 2.1), read as a per-dimension majority;
 *   - Hamming distance between a query and every class hypervector, with
 *     reduction perforation (start, end, stride) applied to the reduction
 *     over dimensions and the result used unscaled (Sec. 2.2 Listing 1;
 *     Sec. 4.2 "Reduction Perforation");
 *   - argmin over the class distances (Sec. 2.2 Listing 1);
 *   - reduced element types for the encoding (Sec. 4.2 "Element Type
 *     Representation"): bfloat16 and OCP FP8 E4M3 inputs.
 *
 * Conventions (readings where the paper is silent):
 *   - bit value 1 encodes the element -1, bit value 0 encodes +1; a zero
 *     projection (y == 0) binarises to +1;
 *   - bit j of word w of a packed hypervector holds element 64*w + j of the
 *     (possibly perforated) dimension list; unused high bits are 0;
 *   - majority bundling ties (2*count == class size) give +1, an empty class
 *     is all +1;
 *   - argmin ties go to the lowest class index;
 *   - the dimension set of a (start, end, stride) configuration is
 *     S = { start + j*stride : start + j*stride < end }.
 */
#ifndef HDC_ORACLE_H
#define HDC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element types (same numbering as the feature types the tests pass in) */
enum { OR_INT8 = 0, OR_UINT8 = 1, OR_BF16 = 2, OR_FP8_E4M3 = 3, OR_FP32 = 4, OR_FP8_SPLIT = 5 };

/* Round a real value to bfloat16: round to nearest, ties to even, on 8
 * significant bits, binary32 exponent range (subnormals below 2^-126),
 * overflow to +-infinity. */
double or_round_bf16(double v);

/* Round a real value to OCP FP8 E4M3FN: round to nearest, ties to even, on 4
 * significant bits, exponent bias 7 (subnormals below 2^-6, quantum 2^-9),
 * largest finite magnitude 448, saturating to +-448. */
double or_round_e4m3(double v);

/* Value of feature f of row i as the encoder sees it under element type
 * `compute`: the exact feature value (compute = INT8 or FP32), or that value
 * rounded to bfloat16 / E4M3.  FP8_SPLIT (integer features only) writes the
 * integer x as a high part h = 16 * floor(x / 16) plus a low part
 * l = x - h in [0, 16), rounds each part to E4M3 on its own and returns
 * their sum: the reduced element type applied to two halves of the
 * feature (Sec. 4.2, "Element Type Representation"). */
double or_feature(const void *X, int x_type, int64_t ldx, int64_t i, int32_t f, int compute);

/* Number of dimensions in S(start, end, stride). */
int32_t or_dims_count(int32_t start, int32_t end, int32_t stride);

/* Random-projection encoding with binarisation.
 *   y[i][j] = sum_{f<F} x'_{if} * P[S_j][f],  H bit j of row i = (y < 0)
 * where x' is the feature value under `compute`.  The sum is exact: int32
 * for integer features under INT8 (|y| < 2^28 for F <= 2^20), an exact
 * fixed-point accumulator for every floating-point case.  H is [n][ldh]
 * uint64 words, |S| bits per row, pad bits 0. */
void or_encode(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
               const int8_t *P, int32_t D, int64_t ldp, int compute,
               int32_t start, int32_t end, int32_t stride,
               uint64_t *H, int64_t ldh, int threads);

/* The projections themselves, y[i][j] as double, plus absum[i] =
 * sum_f |x'_{if}|, for floating-point tolerance bands.  Both are the exact
 * sums rounded once to the nearest double (ties to even). */
void or_project(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
                const int8_t *P, int32_t D, int64_t ldp, int compute,
                int32_t start, int32_t end, int32_t stride,
                double *Y, double *absum, int threads);

/* Majority bundling by counting: n_k = #{i : label_i = k},
 * cnt[k][d] = #{i in class k : bit d set}, C bit d of class k =
 * (2*cnt[k][d] > n_k).  counts (nullable) receives n_k. */
void or_bundle(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
               const int32_t *labels, int32_t K,
               uint64_t *C, int64_t ldc, int32_t *counts);

/* Second, independent bundling: sum of the bipolar values (+1 / -1) of the
 * class members per dimension; the class element is the sign of the sum with
 * a zero sum giving +1. */
void or_bundle_bipolar(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                       const int32_t *labels, int32_t K,
                       uint64_t *C, int64_t ldc);

/* Hamming distance with reduction perforation, by definition: for every
 * query i and class k, the number of d in S(start, end, stride) at which bit
 * d of Q row i differs from bit d of C row k.  Not rescaled. */
void or_hamming(const uint64_t *Q, int64_t n, int64_t ldq,
                const uint64_t *C, int32_t K, int64_t ldc,
                int32_t start, int32_t end, int32_t stride,
                int32_t *dist, int threads);

/* Second, independent Hamming: xor of the packed words, masked to the bits
 * of S, then a population count per word. */
void or_hamming_popcount(const uint64_t *Q, int64_t n, int64_t ldq,
                         const uint64_t *C, int32_t K, int64_t ldc,
                         int32_t start, int32_t end, int32_t stride,
                         int32_t *dist, int threads);

/* First index of the minimum of each row of dist[n][K]. */
void or_argmin(const int32_t *dist, int64_t n, int32_t K, int32_t *label, int32_t *min_dist);

/* One approximation configuration applied to classification: encode the
 * queries over S = S(start, d_trunc, stride) under `compute`, compare bit j
 * of the query with bit S_j of the (full-D) class hypervectors, argmin.
 * dists (nullable) is [n][K]. */
void or_classify(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
                 const int8_t *P, int32_t D, int64_t ldp, int compute,
                 int32_t start, int32_t d_trunc, int32_t stride,
                 const uint64_t *C, int32_t K, int64_t ldc,
                 int32_t *labels, int32_t *dists, int threads);

/* Evaluate configurations cfg[c] = {d_trunc, stride, start, compute} with
 * or_classify and count the queries whose label equals truth. */
void or_eval_configs(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
                     const int32_t *truth, const int8_t *P, int32_t D, int64_t ldp,
                     const uint64_t *C, int32_t K, int64_t ldc,
                     const int32_t *cfg, int32_t ncfg, int32_t *correct, int threads);

/* Number of OpenMP threads a call with `threads` (<= 0: all) will use. */
/* Retraining (Sec. 5, the TRAIN_ITERATIONS knob of the apps; the update
 * rule is not stated in the paper -- the reading taken here is the usual
 * perceptron-style one, applied to a whole epoch at once):
 *   acc[k][d] = sum over rows i of class k of b_i(d),  b = +1 for bit 0, -1
 *               for bit 1 (the bipolar sum that majority bundling
 *               thresholds);
 *   one epoch, with pred[i] the label the model at the start of the epoch
 *   gives row i: for every row with pred[i] != labels[i],
 *               acc[labels[i]] += b_i and acc[pred[i]] -= b_i;
 *   binarised model: bit d of class k is 1 exactly when acc[k][d] < 0
 *               (zero gives +1, as in bundling).
 * acc is [K][nbits] int32. */
void or_class_acc(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                  const int32_t *labels, int32_t K, int32_t *acc);
int64_t or_retrain_epoch(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                         const int32_t *labels, const int32_t *pred, int32_t K, int32_t *acc);
void or_binarize(const int32_t *acc, int32_t K, int32_t nbits, uint64_t *C, int64_t ldc);

/* ADC-chunked dot-product similarity (Sec. 3, in-memory accelerator knobs
 * (I) ADC resolution and (III) analog quantisation scale; Sec. 6 SpecPCM:
 * dot products over 128-element array chunks, each partial product
 * quantised by the ADC before accumulation).  Reading of the unstated
 * quantiser: with the partial s_c = sum over d in chunk c (dimensions
 * [128c, 128c+128)) and in S of b_q(d) * b_k(d) (bipolar +-1),
 *   x = min(max(s_c, floor), ceil),
 *   code = min(floor((x - floor) / step + 1/2), 2^res - 1),
 *   value = floor + step * code;
 * score[i][k] = sum_c value_c over the chunks that hold at least one
 * dimension of S (a chunk with none is not converted), label = first class
 * with the largest score. */
int32_t or_adc_quantize(int32_t s, int32_t res, int32_t step, int32_t floor_, int32_t ceil_);
void or_adc_scores(const uint64_t *Q, int64_t n, int64_t ldq,
                   const uint64_t *C, int32_t K, int64_t ldc,
                   int32_t start, int32_t end, int32_t stride,
                   int32_t res, int32_t step, int32_t floor_, int32_t ceil_,
                   int32_t *scores, int threads);
void or_argmax(const int32_t *scores, int64_t n, int32_t K, int32_t *label, int32_t *max_score);

/* Cosine similarity against non-binarised class hypervectors (Sec. 3
 * "Algorithmic Choice": cosine similarity is the costly alternative to the
 * Hamming distance; the apps' baselines use it).  Reading: the query is the
 * binarised (bipolar) encoding, the class vectors are the integer
 * accumulators acc[K][lda] (bipolar class sums, possibly retrained); over
 * the dimensions S,
 *   dot[k]   = sum over d in S of b_q(d) * acc[k][d]            (exact)
 *   rinv[k]  = 1 / sqrt(sum over d in S of acc[k][d]^2), 0 if that is 0
 *   score[k] = (double)dot[k] * rinv[k]
 * (the query's norm sqrt|S| is the same for every class and is left out);
 * label = first class with the largest score. */
void or_cosine_scores(const uint64_t *Q, int64_t n, int64_t ldq,
                      const int32_t *acc, int32_t K, int64_t lda,
                      int32_t start, int32_t end, int32_t stride,
                      double *scores, int threads);
void or_argmax_f64(const double *scores, int64_t n, int32_t K, int32_t *label, double *max_score);

/* Random-projection encoding with the encoding's own reduction (over the
 * features) perforated (Sec. 4.2 "Reduction Perforation": a perforated
 * matrix-vector product is rescaled for the skipped iterations).  With
 * S_F = { fstart + m*fstride : < fend } and nf = |S_F|,
 *   y[i][j] = (F / nf) * sum over f in S_F of x'_{if} * P[S_j][f],
 * binarised as in or_encode (y < 0 -> bit 1, y == 0 -> +1).  The sum is
 * exact, so the sign of y is exactly the sign of the rescaled value. */
void or_encode_fperf(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
                     const int8_t *P, int32_t D, int64_t ldp, int compute,
                     int32_t fstart, int32_t fend, int32_t fstride,
                     int32_t start, int32_t end, int32_t stride,
                     uint64_t *H, int64_t ldh, int threads);

/* Level-ID encoding (Sec. 3 "Algorithmic Choice": ID-based encoding as the
 * alternative to random projection; Sec. 5.3: the Level knob, the number of
 * discrete levels continuous features are quantised to).  Reading: feature
 * f of row i is quantised to a level, in binary32 arithmetic with every
 * operation rounded to nearest even and nothing fused,
 *   t = x - lo[f];  w = hi[f] - lo[f];  u = t * L;  v = u / w;
 *   level = 0 if !(w > 0) or !(v > 0) (NaN included), L - 1 if v >= L - 1,
 *           else floor(v);
 * and the row's hypervector is the bundle of the bound pairs
 *   s[i][d] = sum over f < F of b(ID_f, d) * b(LV_level(i,f), d),
 *   bit d of H row i = (s < 0)   (s == 0 gives +1),
 * with b(row, d) = +1 for bit 0, -1 for bit 1.  ID [F][ldid] and
 * LV [L][ldlv] are packed hypervectors of D bits (the random identity and
 * level hypervectors are inputs); lev is [n][ldl] uint16.  Multiplying
 * by L before dividing keeps grid points exact: x = lo + k*(hi-lo)/L with
 * an exact product lands on level k. */
void or_level_quantize(const float *X, int64_t n, int32_t F, int64_t ldx,
                       const float *lo, const float *hi, int32_t L,
                       uint16_t *lev, int64_t ldl);
void or_level_id_encode(const uint16_t *lev, int64_t n, int32_t F, int64_t ldl,
                        const uint64_t *ID, int64_t ldid, const uint64_t *LV, int32_t L, int64_t ldlv,
                        int32_t D, uint64_t *H, int64_t ldh, int threads);

int or_threads(int threads);

#ifdef __cplusplus
}
#endif
#endif
