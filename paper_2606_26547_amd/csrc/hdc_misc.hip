// Hamming-distance argmin over packed hypervectors, majority bundling,
// the class-operand tables of the fused classifier and the feature
// conversion diagnostic.
#include <limits.h>

#include "hdc_device.h"

namespace hdc {

// ---------------------------------------------------------------------------
// Class operand table for the fused classifier.  For chunk c (dimensions
// S_{32c .. 32c+31}), class tile kt and lane l, the 16 bytes are the +-1
// values of class kt*32 + l%32 at the dimensions that the encoder's sign
// bytes occupy in lane l: byte b <-> dimension 32c + 8*(b/4) + 4*(l/32) + b%4.
// Classes >= K and dimensions >= nd are 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_class_table(const uint64_t *__restrict__ C, int K, int64_t ldc,
                                                     int s0, int stride, int nd, int KT, int64_t total,
                                                     int8_t *__restrict__ tab)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total)
        return;
    const int lane = (int)(idx & 63);
    const int kt = (int)((idx >> 6) % KT);
    const int64_t c = (idx >> 6) / KT;
    const int k = kt * 32 + (lane & 31), g = lane >> 5;
    uint32_t out[4] = {0, 0, 0, 0};
    if (k < K) {
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const int64_t dl = c * kDimChunk + 8 * (b >> 2) + 4 * g + (b & 3);
            if (dl < nd) {
                const int64_t d = s0 + dl * stride;
                const uint32_t bit = (uint32_t)(C[k * ldc + (d >> 6)] >> (d & 63)) & 1u;
                out[b >> 2] |= (bit ? 0xffu : 0x01u) << (8 * (b & 3));
            }
        }
    }
    *(uint4 *)(tab + idx * 16) = make_uint4(out[0], out[1], out[2], out[3]);
}

// popc[k] = number of -1 elements of class k over S (0 for k >= K).
__global__ __launch_bounds__(256) void k_class_popc(const uint64_t *__restrict__ C, int K, int64_t ldc,
                                                    int s0, int stride, int nd, int32_t *__restrict__ popc)
{
    __shared__ int part[256];
    const int k = blockIdx.x;
    int s = 0;
    if (k < K)
        for (int64_t dl = threadIdx.x; dl < nd; dl += 256) {
            const int64_t d = s0 + dl * stride;
            s += (int)((C[k * ldc + (d >> 6)] >> (d & 63)) & 1u);
        }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        popc[k] = part[0];
}

hipError_t launch_class_popc(const uint64_t *C, int K, int64_t ldc, int s0, int stride, int nd, int KT,
                             int32_t *cpop, hipStream_t st)
{
    hipLaunchKernelGGL(k_class_popc, dim3(KT * 32), dim3(256), 0, st, C, K, ldc, s0, stride, nd, cpop);
    return hipGetLastError();
}

hipError_t launch_class_table(const uint64_t *C, int K, int64_t ldc, int s0, int stride, int nd,
                              int8_t *tab, int32_t *cpop, hipStream_t st)
{
    const int KT = class_tiles(K);
    const int64_t total = table_chunks(nd) * KT * 64;
    hipLaunchKernelGGL(k_class_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, C, K, ldc,
                       s0, stride, nd, KT, total, tab);
    hipLaunchKernelGGL(k_class_popc, dim3(KT * 32), dim3(256), 0, st, C, K, ldc, s0, stride, nd, cpop);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hamming distance + argmin over packed hypervectors (unfused path).  One
// query per lane.  Per window of 16 words the workgroup stages (a) each
// wave's 64 query rows with coalesced 16-byte loads and (b) the 16 words of
// every class, already ANDed with the perforation mask, into LDS; the inner
// loop is branch-free: the query word is masked once, every class word is an
// LDS broadcast read, and each (class, word) costs 2 xor + 2 popcount-
// accumulate.  Classes are compiled in buckets of KB (rows K..KB-1 are zero
// and their distances are ignored); words past the end are zero.
// ---------------------------------------------------------------------------
constexpr int kHamWin = 16;
constexpr int kHamMaxWords = 1024;   // hypervectors up to 65536 bits

template <int KB>
__global__ __launch_bounds__(256) void k_hamming(const uint64_t *__restrict__ Q, int64_t n, int64_t ldq,
                                                 const uint64_t *__restrict__ C, int K, int64_t ldc,
                                                 int start, int end, int stride, int32_t *__restrict__ argmin,
                                                 int32_t *__restrict__ min_dist, int32_t *__restrict__ dists)
{
    __shared__ uint64_t qs[kWaves][64][kHamWin + 1];
    __shared__ uint64_t cls[KB][kHamWin];
    __shared__ uint64_t msk[kHamMaxWords];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int w_lo = start >> 6, w_hi = (end + 63) >> 6;
    for (int w = w_lo + t; w < w_hi; w += 256) {
        uint64_t m = 0;
        const int64_t lo = (int64_t)w * 64 > start ? (int64_t)w * 64 : start;
        const int64_t hi = (int64_t)w * 64 + 64 < end ? (int64_t)w * 64 + 64 : end;
        int64_t d = start + ((lo - start + stride - 1) / stride) * (int64_t)stride;
        for (; d < hi; d += stride)
            m |= 1ull << (d & 63);
        msk[w - w_lo] = m;
    }

    const int64_t rbase = (int64_t)blockIdx.x * 256 + wave * 64;
    int dist[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k)
        dist[k] = 0;

    for (int w0 = w_lo; w0 < w_hi; w0 += kHamWin) {
        __syncthreads();   // masks ready / previous window consumed
        // query tile: 64 rows x 16 words, 16 lanes per row, 4 rows per pass
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            const int r = 4 * p + (lane >> 4), ww = lane & 15;
            const int64_t row = rbase + r;
            uint64_t v = 0;
            if (row < n && w0 + ww < w_hi)
                v = Q[row * ldq + w0 + ww];
            qs[wave][r][ww] = v;
        }
        // class window, masked by S
        for (int i = t; i < KB * kHamWin; i += 256) {
            const int k = i / kHamWin, ww = i % kHamWin;
            uint64_t v = 0;
            if (k < K && w0 + ww < w_hi)
                v = C[(int64_t)k * ldc + w0 + ww] & msk[w0 + ww - w_lo];
            cls[k][ww] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int ww = 0; ww < kHamWin; ++ww) {
            const uint64_t m = (w0 + ww < w_hi) ? msk[w0 + ww - w_lo] : 0ull;
            const uint64_t q = qs[wave][lane][ww] & m;
            const uint32_t ql = (uint32_t)q, qh = (uint32_t)(q >> 32);
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const uint64_t c = cls[k][ww];
                dist[k] += __popc(ql ^ (uint32_t)c) + __popc(qh ^ (uint32_t)(c >> 32));
            }
        }
    }

    const int64_t row = rbase + lane;
    if (row >= n)
        return;
    int bd = INT_MAX, bk = 0;
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (k < K) {
            if (dist[k] < bd) { bd = dist[k]; bk = k; }
            if (dists)
                dists[row * K + k] = dist[k];
        }
    argmin[row] = bk;
    if (min_dist)
        min_dist[row] = bd;
}

#define HDC_HAM_CASE(KB_)                                                                                      \
    if (K <= KB_) {                                                                                            \
        hipLaunchKernelGGL(k_hamming<KB_>, grid, block, 0, st, Q, n, ldq, C, K, ldc, start, end, stride, argmin, \
                           min_dist, dists);                                                                   \
        return hipGetLastError();                                                                              \
    }

hipError_t launch_hamming(const uint64_t *Q, int64_t n, int64_t ldq, const uint64_t *C, int K, int64_t ldc,
                          int start, int end, int stride, int32_t *argmin, int32_t *min_dist,
                          int32_t *dists, hipStream_t st)
{
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    HDC_HAM_CASE(4)
    HDC_HAM_CASE(8)
    HDC_HAM_CASE(12)
    HDC_HAM_CASE(16)
    HDC_HAM_CASE(20)
    HDC_HAM_CASE(24)
    HDC_HAM_CASE(28)
    HDC_HAM_CASE(32)
    HDC_HAM_CASE(48)
    HDC_HAM_CASE(64)
    HDC_HAM_CASE(100)
    HDC_HAM_CASE(128)
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Feature conversion diagnostic: the value of each feature as the encoder's
// X loader converts it (same helpers).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_convert(const void *__restrict__ X, int x_type, int64_t n, int F,
                                                 int64_t ldx, int compute, float *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * F)
        return;
    const int64_t i = idx / F;
    const int f = (int)(idx % F);
    float v;
    if (x_type == X_FP32)
        v = ((const float *)X)[i * ldx + f];
    else {
        const uint32_t b = ((const uint8_t *)X)[i * ldx + f];
        v = byte_value(b, 0, x_type == X_INT8);
    }
    if (compute == C_FP8 || compute == C_FP8H)
        v = __builtin_amdgcn_cvt_f32_fp8((int)fp8x4(v, 0.f, 0.f, 0.f), 0);
    else if (compute == C_FP8S) {   // integer features: the two E4M3 parts, added back
        uint32_t hi, lo;
        fp8_split4(((const uint8_t *)X)[i * ldx + f], x_type == X_INT8, &hi, &lo);
        v = __builtin_amdgcn_cvt_f32_fp8((int)hi, 0) + __builtin_amdgcn_cvt_f32_fp8((int)lo, 0);
    }
    else if (compute == C_BF16)
        v = __uint_as_float(bf16x2(v, 0.f) << 16);
    out[idx] = v;
}

hipError_t launch_convert(const void *X, int x_type, int64_t n, int F, int64_t ldx, int compute, float *out,
                          hipStream_t st)
{
    const int64_t total = n * F;
    hipLaunchKernelGGL(k_convert, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X, x_type, n, F, ldx,
                       compute, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shifted projection: out[d][f] = P[d][f] + 1 (0 or 2 for +-1 weights) for
// f < F, 0 in the pad columns; as E4M3 bytes (2.0 = 0x40, 0 = 0x00) when
// e4m3 is set.  One thread per 16-byte unit of the output; a unit that
// starts below F reads the same unit of P (in bounds: ldp is a multiple of
// 16 and at least F).  Bytes are handled one at a time, so no carry
// crosses into the next weight.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_shift_projection(const int8_t *__restrict__ P, int D, int F, int64_t ldp,
                                                          bool e4m3, int8_t *__restrict__ out, int64_t ldo)
{
    const int64_t upr = ldo / 16;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)D * upr)
        return;
    const int64_t d = idx / upr;
    const int f0 = (int)(idx % upr) * 16;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (f0 < F) {
        const uint4 v = *(const uint4 *)(P + d * ldp + f0);
        const uint32_t in[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int f = f0 + 4 * e + j;
                const uint32_t s = ((in[e] >> (8 * j)) + 1u) & 0xFFu;   // p + 1
                const uint32_t b = f >= F ? 0u : !e4m3 ? s : (s == 2u ? 0x40u : 0u);
                w[e] |= b << (8 * j);
            }
    }
    *(uint4 *)(out + d * ldo + f0) = make_uint4(w[0], w[1], w[2], w[3]);
}

hipError_t launch_shift_projection(const int8_t *P, int D, int F, int64_t ldp, bool e4m3, int8_t *out,
                                   int64_t ldo, hipStream_t st)
{
    const int64_t total = (int64_t)D * (ldo / 16);
    hipLaunchKernelGGL(k_shift_projection, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, P, D, F, ldp,
                       e4m3, out, ldo);
    return hipGetLastError();
}

}  // namespace hdc
