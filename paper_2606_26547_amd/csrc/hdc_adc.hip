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

#include "hdc_stream.h"

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

// ------------------------------------------------------------ prepared
// The same similarity on the matrix cores.  Each chunk partial s is the
// FP4 product of the bipolar query (+-1.0 nibbles) with the class signs
// (+-1.0, 0 outside S) over the chunk's two words: two 32x32x64 MFMAs into
// a fresh fp32 accumulator (|s| <= 128, exact), then every partial goes
// through the ADC table and adds to an int32 score; chunks with no
// dimension of S (uniform) are skipped.  Streaming as in the prepared
// Hamming search (query words and class operand windows into an LDS ring).
//
// Workspace: the class operand (k_sign_table with codes +-1.0) from the
// chunk-aligned word w_lo = 2*floor(start/128), padded to whole windows,
// then the number of dimensions of S in each chunk (int32).
struct AdcLayout {
    int w_lo, w_hi, nwin, KT;
    size_t off_nc, total;
    AdcLayout(int start, int end, int K)
    {
        w_lo = (start >> 7) * 2;
        w_hi = (end + 63) >> 6;
        nwin = (w_hi - w_lo + kHmWin - 1) / kHmWin;
        KT = class_tiles(K);
        off_nc = (size_t)nwin * kHmWin * KT * 1024;
        total = off_nc + (size_t)nwin * (kHmWin / 2) * 4;
    }
};

size_t adc_workspace_bytes(int start, int end, int K) { return AdcLayout(start, end, K).total; }

__global__ __launch_bounds__(256) void k_adc_chunks(int start, int end, int stride, int c_lo, int nchunk,
                                                    int32_t *__restrict__ nc)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= nchunk)
        return;
    const int64_t lo = (int64_t)(c_lo + c) * 128, hi = lo + 128;
    int cnt = 0;
    if (hi > start && lo < end) {
        const int64_t a = lo > start ? lo : start, b = hi < end ? hi : end;
        const int64_t first = start + (a - start + stride - 1) / stride * (int64_t)stride;
        if (first < b)
            cnt = (int)((b - 1 - first) / stride + 1);
    }
    nc[c] = cnt;
}

hipError_t launch_adc_prepare(const uint64_t *C, int K, int64_t ldc, int start, int end, int stride, uint8_t *ws,
                              hipStream_t st)
{
    const AdcLayout L(start, end, K);
    const int64_t total = (int64_t)L.nwin * kHmWin * L.KT * 64;
    // E2M1 +1.0 / -1.0
    hipLaunchKernelGGL((k_sign_table<0x2u, 0xAu>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, C, K,
                       ldc, start, end, stride, L.w_lo, L.KT, total, (int8_t *)ws);
    const int nchunk = L.nwin * (kHmWin / 2);
    hipLaunchKernelGGL(k_adc_chunks, dim3((unsigned)((nchunk + 255) / 256)), dim3(256), 0, st, start, end, stride,
                       L.w_lo / 2, nchunk, (int32_t *)(ws + L.off_nc));
    return hipGetLastError();
}

template <int KT>
__global__ __launch_bounds__(256) void k_adc_mfma(const uint64_t *__restrict__ Q, int64_t n, int64_t ldq, int K,
                                                  int w_lo, int w_hi, int nwin, const int8_t *__restrict__ tab,
                                                  const int32_t *__restrict__ nc, int res, int step, int floor_,
                                                  int ceil_, int32_t *__restrict__ label,
                                                  int32_t *__restrict__ max_score, int32_t *__restrict__ scores)
{
    typedef HmShape<KT> S;
    constexpr int QT = S::QT, W = S::W, ROWS = S::ROWS, NST = S::NST;
    __shared__ __align__(16) uint8_t smem[NST * S::SB];
    __shared__ int lut[257];
    lds_u8 *L = (lds_u8 *)smem;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 5;
    const int64_t rbase = (int64_t)blockIdx.x * ROWS;
    const uint64_t *Qwg = Q + rbase * ldq;

    for (int i = t; i < 257; i += 256) {   // value of every partial s in [-128, 128]
        const int s = i - 128;
        const int64_t x = s < floor_ ? floor_ : (s > ceil_ ? ceil_ : s);
        int64_t code = (2 * (x - floor_) + step) / (2 * (int64_t)step);
        const int64_t top = (1ll << res) - 1;
        if (code > top)
            code = top;
        lut[i] = (int)(floor_ + step * code);
    }
    __syncthreads();

    int qrow[S::NQL], qhalf[S::NQL];
#pragma unroll
    for (int i = 0; i < S::NQL; ++i) {
        const int j = i * kWaves + wave;
        int r = S::RPL * j + lane / S::U;
        qhalf[i] = hm_slot<KT>(r, lane % S::U);
        if (rbase + r >= n)
            r = (int)(n - 1 - rbase);
        qrow[i] = r;
    }
    auto issue = [&](int v, int st) {
        const int vc = v < nwin ? v : nwin - 1;
        lds_u8 *sq = L + st * S::SB;
#pragma unroll
        for (int i = 0; i < S::NQL; ++i) {
            int w = w_lo + vc * W + 2 * qhalf[i];
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
    constexpr int G = S::NQL + S::NTL;

    v16i sc[KT][QT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int qt = 0; qt < QT; ++qt)
            sc[kt][qt] = v16i{};

#pragma unroll
    for (int v = 0; v < NST - 1; ++v)
        issue(v, v);
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(G * (NST - 2)) : "memory");

    int st = 0;
    for (int v = 0; v < nwin; ++v) {
        issue(v + NST - 1, st == 0 ? NST - 1 : st - 1);
        const lds_u8 *sq = L + st * S::SB;
        const lds_u8 *stb = sq + S::QB;
        v4i qv[QT][S::U];
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            const int r = (wave * QT + qt) * 32 + (lane & 31);
#pragma unroll
            for (int hh = 0; hh < S::U; ++hh)
                qv[qt][hh] = *(const lds_v4i *)(sq + r * (W * 8) + 16 * hm_slot<KT>(r, hh));
        }
#pragma unroll
        for (int cc = 0; cc < W / 2; ++cc) {
            if (nc[v * (W / 2) + cc] == 0)   // uniform: not converted
                continue;
            v8i af[2][KT];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    const v4i a4 = *(const lds_v4i *)(stb + (((2 * cc + h) * KT + kt) * 64 + lane) * 16);
                    af[h][kt] = v8i{a4[0], a4[1], a4[2], a4[3], 0, 0, 0, 0};
                }
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) {
                const v4i u = qv[qt][cc];   // the chunk's two words: dwords 0-1 and 2-3
                const v8i b0 = query_bipolar((uint32_t)(g ? u[1] : u[0]));
                const v8i b1 = query_bipolar((uint32_t)(g ? u[3] : u[2]));
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    v16f part = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[0][kt], b0, v16f{}, 4, 4, 0, 0,
                                                                                0, 0);
                    part = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[1][kt], b1, part, 4, 4, 0, 0, 0, 0);
#pragma unroll
                    for (int e = 0; e < 16; ++e)
                        sc[kt][qt][e] += lut[(int)part[e] + 128];
                }
            }
        }
        asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(G * (NST - 2)) : "memory");
        st = st == NST - 1 ? 0 : st + 1;
    }
    __builtin_amdgcn_s_waitcnt(0);

    // argmax: lane holds query l%32 of each tile and classes 8(v/4)+4g+v%4
#pragma unroll
    for (int qt = 0; qt < QT; ++qt) {
        const int64_t q = rbase + (wave * QT + qt) * 32 + (lane & 31);
        int best = INT_MIN, bk = 0;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int k = kt * 32 + 8 * (e >> 2) + 4 * g + (e & 3);
                if (k < K) {
                    const int val = sc[kt][qt][e];
                    if (val > best) { best = val; bk = k; }
                    if (scores && q < n)
                        scores[q * K + k] = val;
                }
            }
        const int ob = __shfl_xor(best, 32), obk = __shfl_xor(bk, 32);
        if (ob > best || (ob == best && obk < bk)) { best = ob; bk = obk; }
        if (g == 0 && q < n) {
            label[q] = bk;
            if (max_score)
                max_score[q] = best;
        }
    }
}

hipError_t launch_adc_prepared(const uint64_t *Q, int64_t n, int64_t ldq, int K, int start, int end, int res,
                               int step, int floor_, int ceil_, const uint8_t *ws, int32_t *label,
                               int32_t *max_score, int32_t *scores, hipStream_t st)
{
    const AdcLayout L(start, end, K);
    const int8_t *tab = (const int8_t *)ws;
    const int32_t *nc = (const int32_t *)(ws + L.off_nc);
#define HDC_ADCP_CASE(KT_)                                                                                     \
    if (L.KT == KT_) {                                                                                         \
        typedef HmShape<KT_> S;                                                                                \
        constexpr int NW = kHmWin / S::W;                                                                      \
        hipLaunchKernelGGL(k_adc_mfma<KT_>, dim3((unsigned)((n + S::ROWS - 1) / S::ROWS)), dim3(256), 0, st, Q,  \
                           n, ldq, K, L.w_lo, L.w_hi, L.nwin * NW, tab, nc, res, step, floor_, ceil_, label,   \
                           max_score, scores);                                                                 \
        return hipGetLastError();                                                                              \
    }
    HDC_ADCP_CASE(1)
    HDC_ADCP_CASE(2)
    HDC_ADCP_CASE(4)
#undef HDC_ADCP_CASE
    return hipErrorInvalidValue;
}

}  // namespace hdc
