// ADC-chunked dot-product similarity: the similarity an in-memory
// accelerator computes when every 128-element array chunk's partial dot
// product is digitised by an ADC before accumulation.  For query i, class k
// and chunk c (dimensions [128c, 128c+128) that lie in S), the partial of
// the bipolar vectors is s = n_c - 2 * popc((q ^ c_k) & mask), n_c the
// chunk's dimensions in S; the ADC maps s to value(s) (clip to [floor,
// ceil], nearest of 2^res levels floor + step*j, ties up), read from a
// 257-entry table in LDS; score = sum of values, label = first class with
// the largest score.  One query per lane, 16-word windows (8 chunks) of the
// queries and of the masked class words staged through LDS as in the
// Hamming kernel.
#include <limits.h>

#include "hdc_device.h"

namespace hdc {

constexpr int kAdcWin = 16;            // words per window (8 chunks)
constexpr int kAdcMaxWords = 1024;     // hypervectors up to 65536 bits

template <int KB>
__global__ __launch_bounds__(256) void k_adc_argmax(const uint64_t *__restrict__ Q, int64_t n, int64_t ldq,
                                                    const uint64_t *__restrict__ C, int K, int64_t ldc, int start,
                                                    int end, int stride, int res, int step, int floor_, int ceil_,
                                                    int32_t *__restrict__ label, int32_t *__restrict__ max_score,
                                                    int32_t *__restrict__ scores)
{
    __shared__ uint64_t qs[kWaves][64][kAdcWin + 1];
    __shared__ uint64_t cls[KB][kAdcWin];
    __shared__ uint64_t msk[kAdcMaxWords];
    __shared__ int lut[257];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int w_lo = (start >> 7) * 2, w_hi = (end + 63) >> 6;   // chunk-aligned first word
    for (int w = w_lo + t; w < w_hi; w += 256) {
        uint64_t m = 0;
        const int64_t lo = (int64_t)w * 64 > start ? (int64_t)w * 64 : start;
        const int64_t hi = (int64_t)w * 64 + 64 < end ? (int64_t)w * 64 + 64 : end;
        for (int64_t d = start + ((lo - start + stride - 1) / stride) * (int64_t)stride; d < hi; d += stride)
            m |= 1ull << (d & 63);
        msk[w - w_lo] = m;
    }
    for (int i = t; i < 257; i += 256) {   // value of every partial s in [-128, 128]
        const int s = i - 128;
        const int64_t x = s < floor_ ? floor_ : (s > ceil_ ? ceil_ : s);
        int64_t code = (2 * (x - floor_) + step) / (2 * (int64_t)step);
        const int64_t top = (1ll << res) - 1;
        if (code > top)
            code = top;
        lut[i] = (int)(floor_ + step * code);
    }

    const int64_t rbase = (int64_t)blockIdx.x * 256 + wave * 64;
    int sc[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k)
        sc[k] = 0;

    for (int w0 = w_lo; w0 < w_hi; w0 += kAdcWin) {
        __syncthreads();   // masks / table ready, previous window consumed
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            const int r = 4 * p + (lane >> 4), ww = lane & 15;
            const int64_t row = rbase + r;
            uint64_t v = 0;
            if (row < n && w0 + ww < w_hi)
                v = Q[row * ldq + w0 + ww];
            qs[wave][r][ww] = v;
        }
        for (int i = t; i < KB * kAdcWin; i += 256) {
            const int k = i / kAdcWin, ww = i % kAdcWin;
            uint64_t v = 0;
            if (k < K && w0 + ww < w_hi)
                v = C[(int64_t)k * ldc + w0 + ww] & msk[w0 + ww - w_lo];
            cls[k][ww] = v;
        }
        __syncthreads();
        for (int cc = 0; cc < kAdcWin / 2; ++cc) {
            const int wa = w0 + 2 * cc;
            const uint64_t m0 = wa < w_hi ? msk[wa - w_lo] : 0ull;
            const uint64_t m1 = wa + 1 < w_hi ? msk[wa + 1 - w_lo] : 0ull;
            const int nc = __popcll(m0) + __popcll(m1);
            if (nc == 0)   // uniform: a chunk without a dimension of S is not converted
                continue;
            const uint64_t q0 = qs[wave][lane][2 * cc] & m0, q1 = qs[wave][lane][2 * cc + 1] & m1;
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int h = __popcll(q0 ^ cls[k][2 * cc]) + __popcll(q1 ^ cls[k][2 * cc + 1]);
                sc[k] += lut[nc - 2 * h + 128];
            }
        }
    }

    const int64_t row = rbase + lane;
    if (row >= n)
        return;
    int best = INT_MIN, bk = 0;
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (k < K) {
            if (sc[k] > best) { best = sc[k]; bk = k; }
            if (scores)
                scores[row * K + k] = sc[k];
        }
    label[row] = bk;
    if (max_score)
        max_score[row] = best;
}

#define HDC_ADC_CASE(KB_)                                                                                      \
    if (K <= KB_) {                                                                                            \
        hipLaunchKernelGGL(k_adc_argmax<KB_>, grid, block, 0, st, Q, n, ldq, C, K, ldc, start, end, stride, res, \
                           step, floor_, ceil_, label, max_score, scores);                                     \
        return hipGetLastError();                                                                              \
    }

hipError_t launch_adc_argmax(const uint64_t *Q, int64_t n, int64_t ldq, const uint64_t *C, int K, int64_t ldc,
                             int start, int end, int stride, int res, int step, int floor_, int ceil_,
                             int32_t *label, int32_t *max_score, int32_t *scores, hipStream_t st)
{
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    HDC_ADC_CASE(4)
    HDC_ADC_CASE(12)
    HDC_ADC_CASE(28)
    HDC_ADC_CASE(64)
    HDC_ADC_CASE(128)
    return hipErrorInvalidValue;
}

}  // namespace hdc
