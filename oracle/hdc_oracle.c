/*
 * hdc_oracle.c -- plain CPU oracle for the HDC classification hot path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  No code, header
 * or table is shared with the GPU library.  Each function states the passage
 * of the paper (arXiv 2606.26547) it follows; see hdc_oracle.h for the
 * conventions taken where the paper is silent.
 *
 * Parallelism is an OpenMP loop over independent queries only; the
 * arithmetic of each query is the plain definition, in order.
 */
#include "hdc_oracle.h"

#include <assert.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int or_threads(int threads)
{
#ifdef _OPENMP
    return threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Reduced element types (Sec. 4.2, "Element Type Representation").     */
/* Both formats are defined by their precision p (significant bits), the */
/* smallest normal exponent emin and the largest finite value: a real v   */
/* is rounded to the nearest multiple of the quantum 2^(e - p + 1), where */
/* e = max(floor(log2|v|), emin), ties to the even multiple.              */
/* ------------------------------------------------------------------ */
static double round_to_format(double v, int p, int emin, double maxfinite, int saturate)
{
    if (v == 0.0 || !isfinite(v))
        return v;
    double a = fabs(v);
    int ex;
    (void)frexp(a, &ex);            /* a = m * 2^ex with m in [0.5, 1) */
    int lead = ex - 1;              /* exponent of the leading bit */
    if (lead < emin)
        lead = emin;                /* subnormal range: fixed quantum */
    double q = ldexp(1.0, lead - (p - 1));
    double r = nearbyint(a / q) * q;   /* default rounding mode: ties to even */
    if (r > maxfinite)
        r = saturate ? maxfinite : INFINITY;
    return copysign(r, v);
}

double or_round_bf16(double v)
{
    /* bfloat16: 8 significant bits, exponent range of binary32 */
    return round_to_format(v, 8, -126, ldexp(255.0, 120), 0);
}

double or_round_e4m3(double v)
{
    /* OCP E4M3FN: 4 significant bits, bias 7 (emin = -6), max 448 = 1.75*2^8 */
    return round_to_format(v, 4, -6, 448.0, 1);
}

/* FP8_SPLIT: x = h + l with h = 16 * floor(x / 16) and l = x - h, each
 * part rounded to E4M3 on its own, then added back. */
static double split_e4m3(double x)
{
    assert(x == floor(x) && x >= -128.0 && x <= 255.0);
    double h = 16.0 * floor(x / 16.0);
    double l = x - h;
    return or_round_e4m3(h) + or_round_e4m3(l);
}

static double raw_feature(const void *X, int x_type, int64_t ldx, int64_t i, int32_t f)
{
    switch (x_type) {
    case OR_INT8:  return (double)((const int8_t *)X)[i * ldx + f];
    case OR_UINT8: return (double)((const uint8_t *)X)[i * ldx + f];
    case OR_FP32:  return (double)((const float *)X)[i * ldx + f];
    default: assert(!"unsupported feature type"); return 0.0;
    }
}

double or_feature(const void *X, int x_type, int64_t ldx, int64_t i, int32_t f, int compute)
{
    double v = raw_feature(X, x_type, ldx, i, f);
    if (compute == OR_BF16)
        return or_round_bf16(v);
    if (compute == OR_FP8_E4M3)
        return or_round_e4m3(v);
    if (compute == OR_FP8_SPLIT)
        return split_e4m3(v);
    return v;
}

int32_t or_dims_count(int32_t start, int32_t end, int32_t stride)
{
    if (stride < 1 || end <= start)
        return 0;
    return (end - start + stride - 1) / stride;
}

/* ------------------------------------------------------------------ */
/* Exact summation of binary32-representable values: a fixed-point       */
/* integer in base 2^32 digits, value = sum_j dig[j] * 2^(32 j - 149).   */
/* Every binary32 value is m * 2^e with integer |m| < 2^24, e >= -149.   */
/* ------------------------------------------------------------------ */
#define XDIG 12
typedef struct { int64_t dig[XDIG]; } xacc;

static void xacc_add(xacc *a, double v)
{
    if (v == 0.0)
        return;
    assert(isfinite(v) && (double)(float)v == v);
    int ex;
    double fr = frexp(fabs(v), &ex);
    int64_t m = (int64_t)ldexp(fr, 53);     /* exact: |v| = m * 2^(ex - 53) */
    int e = ex - 53;
    while ((m & 1) == 0) { m >>= 1; e++; }
    assert(m < (1LL << 24) && e >= -149);
    int shift = e + 149;
    int j = shift / 32, r = shift % 32;
    uint64_t w = (uint64_t)m << r;          /* < 2^56 */
    int64_t lo = (int64_t)(w & 0xffffffffULL), hi = (int64_t)(w >> 32);
    if (v < 0) { lo = -lo; hi = -hi; }
    a->dig[j] += lo;
    a->dig[j + 1] += hi;
}

static void xacc_normalize(xacc *a)
{
    for (int j = 0; j < XDIG - 1; j++) {
        int64_t c = a->dig[j] >> 32;        /* floor(dig / 2^32) */
        a->dig[j] -= c * 4294967296LL;
        a->dig[j + 1] += c;
    }
}

static int xacc_sign(xacc *a)
{
    xacc_normalize(a);
    if (a->dig[XDIG - 1] < 0) return -1;
    for (int j = XDIG - 1; j >= 0; j--)
        if (a->dig[j] != 0) return 1;
    return 0;
}

/* The exact sum rounded once to the nearest double (ties to even): the
 * magnitude's top 96 bits plus a sticky bit for everything below them. */
static double xacc_value(xacc *a)
{
    xacc m = *a;
    xacc_normalize(&m);
    int neg = m.dig[XDIG - 1] < 0;
    if (neg) {
        for (int j = 0; j < XDIG; j++)
            m.dig[j] = -m.dig[j];
        xacc_normalize(&m);
    }
    int t = XDIG - 1;
    while (t >= 0 && m.dig[t] == 0)
        t--;
    if (t < 0)
        return 0.0;
    assert(m.dig[t] > 0 && m.dig[t] < 4294967296LL);
    unsigned __int128 v = 0;
    for (int j = t; j >= t - 2; j--)
        v = (v << 32) | (unsigned __int128)(j >= 0 ? (uint64_t)m.dig[j] : 0);
    int sticky = 0;
    for (int j = t - 3; j >= 0; j--)
        sticky |= m.dig[j] != 0;
    int e0 = 32 * (t - 2) - 149;            /* exponent of bit 0 of v */
    int nb = 0;
    for (unsigned __int128 u = v; u; u >>= 1)
        nb++;
    if (nb > 53) {
        int sh = nb - 53;
        unsigned __int128 rem = v & (((unsigned __int128)1 << sh) - 1);
        unsigned __int128 half = (unsigned __int128)1 << (sh - 1);
        v >>= sh;
        e0 += sh;
        if (rem > half || (rem == half && (sticky || (v & 1))))
            v++;
    }
    double r = ldexp((double)(uint64_t)v, e0);
    return neg ? -r : r;
}

/* Integer features under an element type map to integer values (bfloat16
 * and E4M3 round integers of magnitude <= 255 to integers), so the sum is
 * exact in int32; this builds that map for the 256 possible inputs. */
static int int_feature_table(int x_type, int compute, int32_t tab[256])
{
    if (x_type != OR_INT8 && x_type != OR_UINT8)
        return 0;
    for (int b = 0; b < 256; b++) {
        double raw = x_type == OR_INT8 ? (double)(int8_t)b : (double)b;
        double v = compute == OR_BF16 ? or_round_bf16(raw)
                 : compute == OR_FP8_E4M3 ? or_round_e4m3(raw)
                 : compute == OR_FP8_SPLIT ? split_e4m3(raw) : raw;
        if (v != floor(v))
            return 0;
        tab[b] = (int32_t)v;
    }
    return 1;
}

/* y = sum_f x'_f * P[d][f] for one (row, dimension); returns its sign, and
 * the value through *yv when requested. */
static int project_one(const void *X, int x_type, int64_t ldx, int64_t i, int32_t F,
                       const int8_t *Prow, int compute, const int32_t *tab, double *yv)
{
    if (tab) {
        const uint8_t *x = (const uint8_t *)X + i * ldx;
        int32_t y = 0;
        for (int32_t f = 0; f < F; f++)
            y += tab[x[f]] * (int32_t)Prow[f];
        if (yv) *yv = (double)y;
        return (y > 0) - (y < 0);
    }
    xacc a;
    memset(&a, 0, sizeof a);
    for (int32_t f = 0; f < F; f++)
        xacc_add(&a, or_feature(X, x_type, ldx, i, f, compute) * (double)Prow[f]);
    if (yv) *yv = xacc_value(&a);
    return xacc_sign(&a);
}

/* Random-projection encoding followed by binarisation (Sec. 2.2 Listing 1,
 * the matmul primitive; Sec. 4.2 "Automatic Binarization"). */
void or_encode(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
               const int8_t *P, int32_t D, int64_t ldp, int compute,
               int32_t start, int32_t end, int32_t stride,
               uint64_t *H, int64_t ldh, int threads)
{
    assert(F <= (1 << 20) && end <= D);
    int32_t ns = or_dims_count(start, end, stride);
    int64_t W = (ns + 63) / 64;
    int32_t tab[256];
    int use_tab = int_feature_table(x_type, compute, tab);
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        uint64_t *h = H + i * ldh;
        memset(h, 0, (size_t)W * sizeof(uint64_t));
        for (int32_t j = 0; j < ns; j++) {
            int64_t d = start + (int64_t)j * stride;
            int s = project_one(X, x_type, ldx, i, F, P + d * ldp, compute,
                                use_tab ? tab : NULL, NULL);
            if (s < 0)                      /* -1 -> bit 1; y == 0 -> +1 */
                h[j / 64] |= 1ULL << (j % 64);
        }
    }
}

void or_project(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
                const int8_t *P, int32_t D, int64_t ldp, int compute,
                int32_t start, int32_t end, int32_t stride,
                double *Y, double *absum, int threads)
{
    assert(end <= D);
    int32_t ns = or_dims_count(start, end, stride);
    int32_t tab[256];
    int use_tab = int_feature_table(x_type, compute, tab);
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        xacc s;
        memset(&s, 0, sizeof s);
        for (int32_t f = 0; f < F; f++)
            xacc_add(&s, fabs(or_feature(X, x_type, ldx, i, f, compute)));
        absum[i] = xacc_value(&s);
        for (int32_t j = 0; j < ns; j++) {
            int64_t d = start + (int64_t)j * stride;
            project_one(X, x_type, ldx, i, F, P + d * ldp, compute,
                        use_tab ? tab : NULL, &Y[i * ns + j]);
        }
    }
}

static inline int get_bit(const uint64_t *row, int64_t d)
{
    return (int)((row[d / 64] >> (d % 64)) & 1ULL);
}

/* Class bundling (Sec. 2.1: same-class hypervectors aggregated into a
 * class hypervector), read as the per-dimension majority. */
void or_bundle(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
               const int32_t *labels, int32_t K,
               uint64_t *C, int64_t ldc, int32_t *counts)
{
    int64_t *cnt = calloc((size_t)K * nbits, sizeof(int64_t));
    int64_t *nk = calloc((size_t)K, sizeof(int64_t));
    assert(cnt && nk);
    for (int64_t i = 0; i < n; i++) {
        int32_t k = labels[i];
        assert(k >= 0 && k < K);
        nk[k]++;
        for (int32_t d = 0; d < nbits; d++)
            cnt[(int64_t)k * nbits + d] += get_bit(H + i * ldh, d);
    }
    int64_t W = (nbits + 63) / 64;
    for (int32_t k = 0; k < K; k++) {
        uint64_t *c = C + (int64_t)k * ldc;
        memset(c, 0, (size_t)W * sizeof(uint64_t));
        for (int32_t d = 0; d < nbits; d++)
            if (2 * cnt[(int64_t)k * nbits + d] > nk[k])
                c[d / 64] |= 1ULL << (d % 64);
        if (counts)
            counts[k] = (int32_t)nk[k];
    }
    free(cnt);
    free(nk);
}

void or_bundle_bipolar(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                       const int32_t *labels, int32_t K,
                       uint64_t *C, int64_t ldc)
{
    int64_t *sum = calloc((size_t)K * nbits, sizeof(int64_t));
    assert(sum);
    for (int64_t i = 0; i < n; i++)
        for (int32_t d = 0; d < nbits; d++)
            sum[(int64_t)labels[i] * nbits + d] += get_bit(H + i * ldh, d) ? -1 : +1;
    int64_t W = (nbits + 63) / 64;
    for (int32_t k = 0; k < K; k++) {
        uint64_t *c = C + (int64_t)k * ldc;
        memset(c, 0, (size_t)W * sizeof(uint64_t));
        for (int32_t d = 0; d < nbits; d++)
            if (sum[(int64_t)k * nbits + d] < 0)
                c[d / 64] |= 1ULL << (d % 64);
    }
    free(sum);
}

/* Hamming distance (Sec. 2.2 Listing 1) under reduction perforation
 * (Sec. 4.2): the reduction over dimensions visits only S(start, end,
 * stride); the count is used as-is. */
void or_hamming(const uint64_t *Q, int64_t n, int64_t ldq,
                const uint64_t *C, int32_t K, int64_t ldc,
                int32_t start, int32_t end, int32_t stride,
                int32_t *dist, int threads)
{
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++)
        for (int32_t k = 0; k < K; k++) {
            int32_t s = 0;
            for (int64_t d = start; d < end; d += stride)
                s += get_bit(Q + i * ldq, d) != get_bit(C + (int64_t)k * ldc, d);
            dist[i * K + k] = s;
        }
}

void or_hamming_popcount(const uint64_t *Q, int64_t n, int64_t ldq,
                         const uint64_t *C, int32_t K, int64_t ldc,
                         int32_t start, int32_t end, int32_t stride,
                         int32_t *dist, int threads)
{
    int64_t W = (end + 63) / 64;
    uint64_t *mask = calloc((size_t)(W > 0 ? W : 1), sizeof(uint64_t));
    assert(mask);
    for (int64_t d = start; d < end; d += stride)
        mask[d / 64] |= 1ULL << (d % 64);
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++)
        for (int32_t k = 0; k < K; k++) {
            int32_t s = 0;
            for (int64_t w = 0; w < W; w++)
                s += __builtin_popcountll((Q[i * ldq + w] ^ C[(int64_t)k * ldc + w]) & mask[w]);
            dist[i * K + k] = s;
        }
    free(mask);
}

/* argmin over classes (Sec. 2.2 Listing 1), first minimum on ties. */
void or_argmin(const int32_t *dist, int64_t n, int32_t K, int32_t *label, int32_t *min_dist)
{
    for (int64_t i = 0; i < n; i++) {
        int32_t best = 0;
        for (int32_t k = 1; k < K; k++)
            if (dist[i * K + k] < dist[i * K + best])
                best = k;
        label[i] = best;
        if (min_dist)
            min_dist[i] = dist[i * K + best];
    }
}

/* Inference under one approximation configuration: encoding over the
 * dimensions S (Sec. 4.2 "Encoding Dimensionality" / reduction
 * perforation), Hamming distance of bit j of the query against bit S_j of
 * each class hypervector, argmin. */
void or_classify(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
                 const int8_t *P, int32_t D, int64_t ldp, int compute,
                 int32_t start, int32_t d_trunc, int32_t stride,
                 const uint64_t *C, int32_t K, int64_t ldc,
                 int32_t *labels, int32_t *dists, int threads)
{
    int32_t ns = or_dims_count(start, d_trunc, stride);
    int64_t W = (ns + 63) / 64;
    if (W == 0) W = 1;
    uint64_t *Hq = calloc((size_t)(n > 0 ? n : 1) * W, sizeof(uint64_t));
    int32_t *dd = dists ? dists : malloc((size_t)(n > 0 ? n : 1) * K * sizeof(int32_t));
    assert(Hq && dd);
    or_encode(X, x_type, n, F, ldx, P, D, ldp, compute, start, d_trunc, stride, Hq, W, threads);
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++)
        for (int32_t k = 0; k < K; k++) {
            int32_t s = 0;
            for (int32_t j = 0; j < ns; j++)
                s += get_bit(Hq + i * W, j) != get_bit(C + (int64_t)k * ldc, start + (int64_t)j * stride);
            dd[i * K + k] = s;
        }
    or_argmin(dd, n, K, labels, NULL);
    if (!dists)
        free(dd);
    free(Hq);
}

void or_eval_configs(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
                     const int32_t *truth, const int8_t *P, int32_t D, int64_t ldp,
                     const uint64_t *C, int32_t K, int64_t ldc,
                     const int32_t *cfg, int32_t ncfg, int32_t *correct, int threads)
{
    int32_t *lab = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    assert(lab);
    for (int32_t c = 0; c < ncfg; c++) {
        const int32_t *g = cfg + 4 * c;     /* d_trunc, stride, start, compute */
        or_classify(X, x_type, n, F, ldx, P, D, ldp, g[3], g[2], g[0], g[1],
                    C, K, ldc, lab, NULL, threads);
        int32_t ok = 0;
        for (int64_t i = 0; i < n; i++)
            ok += lab[i] == truth[i];
        correct[c] = ok;
    }
    free(lab);
}

/* ------------------------------------------------------------------------
 * Retraining: integer class accumulators and one epoch of mispredicted-row
 * updates (see the header for the reading of the rule).
 * ---------------------------------------------------------------------- */
static int32_t bipolar(const uint64_t *h, int32_t d)
{
    return get_bit(h, d) ? -1 : 1;
}

void or_class_acc(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                  const int32_t *labels, int32_t K, int32_t *acc)
{
    memset(acc, 0, (size_t)K * nbits * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) {
        int32_t k = labels[i];
        assert(k >= 0 && k < K);
        for (int32_t d = 0; d < nbits; d++)
            acc[(int64_t)k * nbits + d] += bipolar(H + i * ldh, d);
    }
}

int64_t or_retrain_epoch(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                         const int32_t *labels, const int32_t *pred, int32_t K, int32_t *acc)
{
    int64_t wrong = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t y = labels[i], p = pred[i];
        assert(y >= 0 && y < K && p >= 0 && p < K);
        if (p == y)
            continue;
        wrong++;
        for (int32_t d = 0; d < nbits; d++) {
            int32_t b = bipolar(H + i * ldh, d);
            acc[(int64_t)y * nbits + d] += b;
            acc[(int64_t)p * nbits + d] -= b;
        }
    }
    return wrong;
}

void or_binarize(const int32_t *acc, int32_t K, int32_t nbits, uint64_t *C, int64_t ldc)
{
    int64_t W = (nbits + 63) / 64;
    for (int32_t k = 0; k < K; k++) {
        uint64_t *c = C + (int64_t)k * ldc;
        memset(c, 0, (size_t)W * sizeof(uint64_t));
        for (int32_t d = 0; d < nbits; d++)
            if (acc[(int64_t)k * nbits + d] < 0)
                c[d / 64] |= 1ULL << (d % 64);
    }
}

/* ------------------------------------------------------------------------
 * ADC-chunked similarity (see the header for the reading of the quantiser).
 * ---------------------------------------------------------------------- */
int32_t or_adc_quantize(int32_t s, int32_t res, int32_t step, int32_t floor_, int32_t ceil_)
{
    int64_t x = s < floor_ ? floor_ : (s > ceil_ ? ceil_ : s);
    /* floor((x - floor) / step + 1/2) with x - floor >= 0 */
    int64_t code = (2 * (x - floor_) + step) / (2 * (int64_t)step);
    int64_t top = (1LL << res) - 1;
    if (code > top)
        code = top;
    return (int32_t)(floor_ + step * code);
}

void or_adc_scores(const uint64_t *Q, int64_t n, int64_t ldq,
                   const uint64_t *C, int32_t K, int64_t ldc,
                   int32_t start, int32_t end, int32_t stride,
                   int32_t res, int32_t step, int32_t floor_, int32_t ceil_,
                   int32_t *scores, int threads)
{
    int64_t nchunks = (end + 127) / 128;
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++)
        for (int32_t k = 0; k < K; k++) {
            int32_t total = 0;
            for (int64_t c = 0; c < nchunks; c++) {
                int32_t sc = 0, used = 0;
                for (int64_t d = 128 * c; d < 128 * c + 128 && d < end; d++) {
                    if (d < start || (d - start) % stride != 0)
                        continue;
                    int32_t bq = get_bit(Q + i * ldq, d) ? -1 : 1;
                    int32_t bk = get_bit(C + (int64_t)k * ldc, d) ? -1 : 1;
                    sc += bq * bk;
                    used++;
                }
                if (used)   /* a chunk with no dimension of S is not converted */
                    total += or_adc_quantize(sc, res, step, floor_, ceil_);
            }
            scores[i * K + k] = total;
        }
}

void or_argmax(const int32_t *scores, int64_t n, int32_t K, int32_t *label, int32_t *max_score)
{
    for (int64_t i = 0; i < n; i++) {
        int32_t best = 0;
        for (int32_t k = 1; k < K; k++)
            if (scores[i * K + k] > scores[i * K + best])
                best = k;
        label[i] = best;
        if (max_score)
            max_score[i] = scores[i * K + best];
    }
}

/* ------------------------------------------------------------------------
 * Cosine similarity against integer class accumulators (see the header).
 * ---------------------------------------------------------------------- */
void or_cosine_scores(const uint64_t *Q, int64_t n, int64_t ldq,
                      const int32_t *acc, int32_t K, int64_t lda,
                      int32_t start, int32_t end, int32_t stride,
                      double *scores, int threads)
{
    double *rinv = malloc((size_t)K * sizeof(double));
    assert(rinv);
    for (int32_t k = 0; k < K; k++) {
        int64_t nsq = 0;
        for (int64_t d = start; d < end; d += stride)
            nsq += (int64_t)acc[k * lda + d] * acc[k * lda + d];
        rinv[k] = nsq > 0 ? 1.0 / sqrt((double)nsq) : 0.0;
    }
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++)
        for (int32_t k = 0; k < K; k++) {
            int64_t dot = 0;
            for (int64_t d = start; d < end; d += stride)
                dot += (int64_t)(get_bit(Q + i * ldq, d) ? -1 : 1) * acc[k * lda + d];
            scores[i * K + k] = (double)dot * rinv[k];
        }
    free(rinv);
}

void or_argmax_f64(const double *scores, int64_t n, int32_t K, int32_t *label, double *max_score)
{
    for (int64_t i = 0; i < n; i++) {
        int32_t best = 0;
        for (int32_t k = 1; k < K; k++)
            if (scores[i * K + k] > scores[i * K + best])
                best = k;
        label[i] = best;
        if (max_score)
            max_score[i] = scores[i * K + best];
    }
}

/* ------------------------------------------------------------------------
 * Encoding with the reduction over features perforated (header: the sign
 * of the rescaled product).
 * ---------------------------------------------------------------------- */
static int project_sub(const void *X, int x_type, int64_t ldx, int64_t i, int32_t fstart, int32_t fend,
                       int32_t fstride, const int8_t *Prow, int compute, const int32_t *tab)
{
    if (tab) {
        const uint8_t *x = (const uint8_t *)X + i * ldx;
        int32_t y = 0;
        for (int32_t f = fstart; f < fend; f += fstride)
            y += tab[x[f]] * (int32_t)Prow[f];
        return (y > 0) - (y < 0);
    }
    xacc a;
    memset(&a, 0, sizeof a);
    for (int32_t f = fstart; f < fend; f += fstride)
        xacc_add(&a, or_feature(X, x_type, ldx, i, f, compute) * (double)Prow[f]);
    return xacc_sign(&a);
}

void or_encode_fperf(const void *X, int x_type, int64_t n, int32_t F, int64_t ldx,
                     const int8_t *P, int32_t D, int64_t ldp, int compute,
                     int32_t fstart, int32_t fend, int32_t fstride,
                     int32_t start, int32_t end, int32_t stride,
                     uint64_t *H, int64_t ldh, int threads)
{
    assert(F <= (1 << 20) && end <= D && fend <= F);
    int32_t nf = or_dims_count(fstart, fend, fstride);
    assert(nf > 0);
    double scale = (double)F / nf;          /* compensation for skipped terms */
    int scale_sign = (scale > 0) - (scale < 0);
    int32_t ns = or_dims_count(start, end, stride);
    int64_t W = (ns + 63) / 64;
    int32_t tab[256];
    int use_tab = int_feature_table(x_type, compute, tab);
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        uint64_t *h = H + i * ldh;
        memset(h, 0, (size_t)W * sizeof(uint64_t));
        for (int32_t j = 0; j < ns; j++) {
            int64_t d = start + (int64_t)j * stride;
            int s = scale_sign * project_sub(X, x_type, ldx, i, fstart, fend, fstride, P + d * ldp, compute,
                                             use_tab ? tab : NULL);
            if (s < 0)
                h[j / 64] |= 1ULL << (j % 64);
        }
    }
}

/* ------------------------------------------------------------------------
 * Level-ID encoding (header: quantiser and bound-pair bundle).
 * ---------------------------------------------------------------------- */
void or_level_quantize(const float *X, int64_t n, int32_t F, int64_t ldx,
                       const float *lo, const float *hi, int32_t L,
                       uint16_t *lev, int64_t ldl)
{
    assert(L >= 1 && L <= 65536);
    for (int64_t i = 0; i < n; i++)
        for (int32_t f = 0; f < F; f++) {
            volatile float t = X[i * ldx + f] - lo[f];
            volatile float w = hi[f] - lo[f];
            volatile float u = t * (float)L;
            volatile float v = u / w;
            int32_t level;
            if (!(w > 0.0f) || !(v > 0.0f))
                level = 0;
            else if (v >= (float)(L - 1))
                level = L - 1;
            else
                level = (int32_t)floorf(v);
            lev[i * ldl + f] = (uint16_t)level;
        }
}

void or_level_id_encode(const uint16_t *lev, int64_t n, int32_t F, int64_t ldl,
                        const uint64_t *ID, int64_t ldid, const uint64_t *LV, int32_t L, int64_t ldlv,
                        int32_t D, uint64_t *H, int64_t ldh, int threads)
{
    int64_t W = (D + 63) / 64;
#pragma omp parallel for num_threads(or_threads(threads)) schedule(dynamic, 4)
    for (int64_t i = 0; i < n; i++) {
        uint64_t *h = H + i * ldh;
        memset(h, 0, (size_t)W * sizeof(uint64_t));
        for (int32_t d = 0; d < D; d++) {
            int32_t s = 0;
            for (int32_t f = 0; f < F; f++) {
                int32_t l = lev[i * ldl + f];
                assert(l < L);
                int32_t bid = get_bit(ID + (int64_t)f * ldid, d) ? -1 : 1;
                int32_t blv = get_bit(LV + (int64_t)l * ldlv, d) ? -1 : 1;
                s += bid * blv;
            }
            if (s < 0)
                h[d / 64] |= 1ULL << (d % 64);
        }
    }
}
