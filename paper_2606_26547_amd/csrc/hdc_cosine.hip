// Cosine similarity of bipolar query hypervectors against non-binarised
// (integer) class accumulators, on the matrix cores.
//
// With q'_d in {0,1} the query bit (1 = element -1) and a_kd the class
// accumulator, the dot product over S is
//     dot_k = sum_S a_kd - 2 * sum_S q'_d * a_kd.
// The second sum runs as int8 MFMAs (rows = classes, columns = queries,
// K = 32 dimensions): a_kd = 256 * hi + lo with hi, lo in [-128, 127]
// (|a| <= 32639), one MFMA per part; the query operand holds the bits as
// bytes {0, 1}, two operations per register (see spread_bits).
// score_k = (double)dot_k * rinv_k with rinv_k = 1 / sqrt(sum_S a_kd^2)
// (0 for an all-zero class), both roundings correctly rounded, so the
// scores equal a plain double computation bit for bit; label = first class
// with the largest score.  An accumulator entry over S outside [-32639,
// 32639] does not fit the split: _prepare then clears a flag in the
// workspace and every label of the search is -1, every score NaN.
//
// Prepared operand (hdc_cosine_prepare): for word w (from the even word at
// or below the first word of S, padded to whole 8-word windows), dword half
// h, part p (lo, hi) and class tile kt, 64 lanes x 16 bytes: lane l, byte
// b = 4r + i holds part p of a_kd for class kt*32 + l%32 at dimension
// 64w + 32h + 4*(l/32) + r + 8i (0 outside S), the order in which the
// query operand takes the dword's bits (register r of lane half g =
// (dword >> (4g + r)) & 0x01010101); then T_k = sum_S a_kd (int64)
// and rinv_k (double) for 128 classes, max |a_kd| over S per class (int32)
// and the range flag.
//
// Streaming as in the prepared Hamming search: query words and operand
// windows go from global memory straight into a two-stage LDS ring
// (global_load_lds), one barrier per window.
#include <limits.h>

#include "hdc_device.h"

namespace hdc {

template <int KT, int QT_ = (KT == 4 ? 1 : 2), int NST_ = (KT == 1 ? 3 : 2)> struct CosShape {
    static constexpr int QT = QT_;
    static constexpr int W = 4;                        // words per window (divides kCosWin)
    static constexpr int U = W / 2;                    // 16-byte units per query row
    static constexpr int RPL = 64 / U;                 // query rows per 1 KiB load
    static constexpr int ROWS = kWaves * QT * 32;      // queries per workgroup
    static constexpr int QB = ROWS * W * 8;            // query bytes per stage
    static constexpr int TB = W * 4 * KT * 1024;       // operand bytes per window
    static constexpr int NST = NST_;
    static constexpr int NQL = QB / 1024 / kWaves;
    static constexpr int NTL = TB / 1024 / kWaves;
    static constexpr int SB = QB + TB;
};
constexpr int kCosWin = 8;
constexpr int kCosMaxAcc = 32639;   // |a| bound of the two-byte split

struct CosLayout {
    int w_lo, w_hi, nwin, KT;
    size_t off_T, off_rinv, off_amax, off_flag, total;
    CosLayout(int start, int end, int K)
    {
        w_lo = (start >> 6) & ~1;
        w_hi = (end + 63) >> 6;
        nwin = (w_hi - w_lo + kCosWin - 1) / kCosWin;
        KT = class_tiles(K);
        off_T = (size_t)nwin * kCosWin * 4 * KT * 1024;
        off_rinv = off_T + 128 * 8;
        off_amax = off_rinv + 128 * 8;
        off_flag = off_amax + 128 * 4;
        total = off_flag + 16;
    }
};

size_t cos_workspace_bytes(int start, int end, int K) { return CosLayout(start, end, K).total; }

__device__ __forceinline__ bool in_set(int64_t d, int start, int end, int stride)
{
    return d >= start && d < end && (d - start) % stride == 0;
}

__global__ __launch_bounds__(256) void k_cos_table(const int32_t *__restrict__ acc, int K, int64_t lda, int start,
                                                   int end, int stride, int w_lo, int KT, int64_t total,
                                                   int8_t *__restrict__ tab)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total)
        return;
    const int lane = (int)(idx & 63);
    const int kt = (int)((idx >> 6) % KT);
    const int64_t whp = (idx >> 6) / KT;   // (word * 2 + half) * 2 + part
    const int part = (int)(whp & 1);
    const int h = (int)((whp >> 1) & 1);
    const int64_t w = w_lo + (whp >> 2);
    const int k = kt * 32 + (lane & 31), g = lane >> 5;
    uint32_t o[4] = {0, 0, 0, 0};
    if (k < K) {
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const int64_t d = w * 64 + 32 * h + 4 * g + (b >> 2) + 8 * (b & 3);
            if (in_set(d, start, end, stride)) {
                const int a = acc[k * lda + d];
                const int hi = (a + 128) >> 8;
                const int v = part ? hi : a - 256 * hi;
                o[b >> 2] |= ((uint32_t)v & 0xffu) << (8 * (b & 3));
            }
        }
    }
    *(uint4 *)(tab + idx * 16) = make_uint4(o[0], o[1], o[2], o[3]);
}

// T_k, rinv_k and max |a_kd| over S, one workgroup per class (classes past
// K get 0).
__global__ __launch_bounds__(256) void k_cos_norms(const int32_t *__restrict__ acc, int K, int64_t lda, int start,
                                                   int end, int stride, int64_t *__restrict__ T,
                                                   double *__restrict__ rinv, int32_t *__restrict__ amax)
{
    __shared__ long long ps[256], pq[256], pm[256];
    const int k = blockIdx.x, t = threadIdx.x;
    long long s = 0, q = 0, m = 0;
    if (k < K)
        for (int64_t d = start + (int64_t)t * stride; d < end; d += (int64_t)256 * stride) {
            const long long a = acc[k * lda + d];
            s += a;
            q += a * a;
            m = a > m ? a : (-a > m ? -a : m);
        }
    ps[t] = s;
    pq[t] = q;
    pm[t] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            ps[t] += ps[t + h];
            pq[t] += pq[t + h];
            pm[t] = pm[t + h] > pm[t] ? pm[t + h] : pm[t];
        }
        __syncthreads();
    }
    if (t == 0) {
        T[k] = ps[0];
        rinv[k] = pq[0] > 0 ? __ddiv_rn(1.0, __dsqrt_rn((double)pq[0])) : 0.0;
        amax[k] = pm[0] > INT_MAX ? INT_MAX : (int32_t)pm[0];
    }
}

__global__ __launch_bounds__(128) void k_cos_flag(const int32_t *__restrict__ amax, int32_t *__restrict__ flag)
{
    __shared__ int bad;
    if (threadIdx.x == 0)
        bad = 0;
    __syncthreads();
    if (amax[threadIdx.x] > kCosMaxAcc)
        atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0)
        flag[0] = bad ? 0 : 1;
}

// Query bits as bytes {0, 1}: register r of lane half g holds, in byte i,
// bit 4g + r + 8i of the dword (two operations per register).
__device__ __forceinline__ v4i spread_bits(uint32_t d, uint32_t sh)
{
    const uint32_t e = d >> sh;
    v4i b;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        b[r] = (int)((e >> r) & 0x01010101u);
    return b;
}

template <int KT, int QT_, int NST_>
__global__ __launch_bounds__(256) void k_cosine_mfma(const uint64_t *__restrict__ Q, int64_t n, int64_t ldq, int K,
                                                     int w_lo, int w_hi, int nwin, const int8_t *__restrict__ tab,
                                                     const int64_t *__restrict__ T, const double *__restrict__ rinv,
                                                     const int32_t *__restrict__ flag, int32_t *__restrict__ label, double *__restrict__ max_score,
                                                     double *__restrict__ scores)
{
    typedef CosShape<KT, QT_, NST_> S;
    constexpr int QT = S::QT, W = S::W, NST = S::NST;
    constexpr int G = S::NQL + S::NTL;                 // loads per window and wave
    __shared__ __align__(16) uint8_t smem[NST * S::SB];
    lds_u8 *L = (lds_u8 *)smem;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 5;
    const uint32_t sh = 4u * (uint32_t)g;
    const int64_t rbase = (int64_t)blockIdx.x * S::ROWS;
    const uint64_t *Qwg = Q + rbase * ldq;

    // query loads: load i of a wave fills rows RPL*j .. (j = i*4 + wave),
    // lane l -> row RPL*j + l/U, unit l%U of the window (rows past n
    // re-read row n-1; 16-byte units of 2 words, no swizzle needed for the
    // 8-byte reads below)
    int qrow[S::NQL], qunit[S::NQL];
#pragma unroll
    for (int i = 0; i < S::NQL; ++i) {
        const int j = i * kWaves + wave;
        int r = S::RPL * j + lane / S::U;
        qunit[i] = lane % S::U;
        if (rbase + r >= n)
            r = (int)(n - 1 - rbase);
        qrow[i] = r;
    }
    auto issue = [&](int v, int st) {
        const int vc = v < nwin ? v : nwin - 1;
        lds_u8 *sq = L + st * S::SB;
#pragma unroll
        for (int i = 0; i < S::NQL; ++i) {
            int w = w_lo + vc * W + 2 * qunit[i];
            if (w >= w_hi)
                w = w_lo;
            lds_dma16(Qwg, (uint32_t)(((int64_t)qrow[i] * ldq + w) * 8), sq + (i * kWaves + wave) * 1024);
        }
#pragma unroll
        for (int i = 0; i < S::NTL; ++i) {
            const int j = i * kWaves + wave;
            lds_dma16(tab, (uint32_t)(vc * S::TB + j * 1024 + lane * 16), sq + S::QB + j * 1024);
        }
    };

    v16i alo[KT][QT], ahi[KT][QT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            alo[kt][qt] = v16i{};
            ahi[kt][qt] = v16i{};
        }

    // ring of NST stages: window v lives in stage v % NST; loads run NST-1
    // windows ahead, and vector memory operations complete in order, so
    // vmcnt(G*(NST-2)) leaves only the newer windows in flight
#pragma unroll
    for (int v = 0; v < NST - 1; ++v)
        issue(v, v);
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(G * (NST - 2)) : "memory");
    int st = 0;
    for (int v = 0; v < nwin; ++v) {
        issue(v + NST - 1, st == 0 ? NST - 1 : st - 1);
        const lds_u8 *sq = L + st * S::SB;
        const lds_u8 *stb = sq + S::QB;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            uint64_t q[QT];
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) {
                const int r = (wave * QT + qt) * 32 + (lane & 31);
                q[qt] = *(const HDC_LDS uint64_t *)(sq + (r * W + ww) * 8);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                v4i flo[KT], fhi[KT];
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    flo[kt] = *(const lds_v4i *)(stb + ((((ww * 2 + h) * 2 + 0) * KT + kt) * 64 + lane) * 16);
                    fhi[kt] = *(const lds_v4i *)(stb + ((((ww * 2 + h) * 2 + 1) * KT + kt) * 64 + lane) * 16);
                }
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) {
                    const v4i bf = spread_bits(h ? (uint32_t)(q[qt] >> 32) : (uint32_t)q[qt], sh);
#pragma unroll
                    for (int kt = 0; kt < KT; ++kt) {
                        alo[kt][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(flo[kt], bf, alo[kt][qt], 0, 0, 0);
                        ahi[kt][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fhi[kt], bf, ahi[kt][qt], 0, 0, 0);
                    }
                }
            }
        }
        asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(G * (NST - 2)) : "memory");
        st = st == NST - 1 ? 0 : st + 1;
    }
    __builtin_amdgcn_s_waitcnt(0);

    // argmax: lane holds query l%32 of each tile and classes 8(v/4)+4g+v%4
    const bool in_range = flag[0] != 0;
    const double nan = __builtin_nan("");
#pragma unroll
    for (int qt = 0; qt < QT; ++qt) {
        const int64_t q = rbase + (wave * QT + qt) * 32 + (lane & 31);
        double best = -1.0 / 0.0;
        int bk = 0;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int k = kt * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
                if (k < K) {
                    const long long s = 256ll * ahi[kt][qt][v] + alo[kt][qt][v];
                    const double sc = in_range ? __dmul_rn((double)(T[k] - 2 * s), rinv[k]) : nan;
                    if (sc > best) { best = sc; bk = k; }
                    if (scores && q < n)
                        scores[q * K + k] = sc;
                }
            }
        const double ob = __shfl_xor(best, 32);
        const int obk = __shfl_xor(bk, 32);
        if (ob > best || (ob == best && obk < bk)) { best = ob; bk = obk; }
        if (g == 0 && q < n) {
            label[q] = in_range ? bk : -1;
            if (max_score)
                max_score[q] = in_range ? best : nan;
        }
    }
}

hipError_t launch_cos_prepare(const int32_t *acc, int K, int64_t lda, int start, int end, int stride, uint8_t *ws,
                              hipStream_t st)
{
    const CosLayout L(start, end, K);
    const int64_t total = (int64_t)L.nwin * kCosWin * 4 * L.KT * 64;
    hipLaunchKernelGGL(k_cos_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, acc, K, lda, start, end,
                       stride, L.w_lo, L.KT, total, (int8_t *)ws);
    hipLaunchKernelGGL(k_cos_norms, dim3(128), dim3(256), 0, st, acc, K, lda, start, end, stride,
                       (int64_t *)(ws + L.off_T), (double *)(ws + L.off_rinv), (int32_t *)(ws + L.off_amax));
    hipLaunchKernelGGL(k_cos_flag, dim3(1), dim3(128), 0, st, (const int32_t *)(ws + L.off_amax),
                       (int32_t *)(ws + L.off_flag));
    return hipGetLastError();
}

hipError_t launch_cos_prepared(const uint64_t *Q, int64_t n, int64_t ldq, int K, int start, int end,
                               const uint8_t *ws, int32_t *label, double *max_score, double *scores, hipStream_t st)
{
    const CosLayout L(start, end, K);
    const int8_t *tab = (const int8_t *)ws;
    const int64_t *T = (const int64_t *)(ws + L.off_T);
    const double *rinv = (const double *)(ws + L.off_rinv);
    const int32_t *flag = (const int32_t *)(ws + L.off_flag);
#define HDC_COS_CASE(KT_)                                                                                      \
    if (L.KT == KT_) {                                                                                         \
        typedef CosShape<KT_> S;                                                                               \
        constexpr int R = S::ROWS, NW = kCosWin / S::W;                                                        \
        hipLaunchKernelGGL((k_cosine_mfma<KT_, S::QT, S::NST>), dim3((unsigned)((n + R - 1) / R)), dim3(256), 0, \
                           st, Q, n, ldq,                                                                      \
                           K, L.w_lo, L.w_hi, L.nwin * NW, tab, T, rinv, flag, label, max_score, scores);            \
        return hipGetLastError();                                                                              \
    }
    HDC_COS_CASE(1)
    HDC_COS_CASE(2)
    HDC_COS_CASE(4)
#undef HDC_COS_CASE
    return hipErrorInvalidValue;
}

}  // namespace hdc
