// Hamming distance + argmin over packed hypervectors on the matrix cores.
//
// With q'_d in {0,1} the query bit (1 = element -1) and c_d = +1 / -1 the
// class element, the Hamming distance over S is
//     dist = popc_S(c) + sum_{d in S} q'_d * c_d.
// The sum runs as an FP4 (E2M1) MFMA with fp32 accumulation (rows =
// classes, columns = queries, K = 64 dimensions = one query word per
// instruction): the query operand holds 0.5 for a set bit and 0 otherwise,
// the class operand 2.0 * c_d (0 outside S), so every product is exactly
// +-1 or 0 and every partial sum is an integer far below 2^24: the fp32
// accumulator is exact.  Lane half g takes dword g of the word; its register
// r is (dword >> r) & 0x11111111, i.e. nibble j holds bit 4j + r, so one
// shift and one AND per register build the operand.  Dimensions outside S
// (perforated, or past the end) have class nibble 0, so query bits there
// contribute nothing and the queries need no masking.
//
// Class operand table (built once per (classes, perforation) by
// k_sign_table with codes +-2.0): for word w (counted from the even word w_lo at or below the
// first word of S, padded with zero words to whole windows) and class tile
// kt, 64 lanes x 16 bytes where lane l, nibble j of dword r holds class
// kt*32 + l%32 at dimension 64w + 32*(l/32) + 4j + r.
//
// Streaming: a workgroup (4 waves, one per SIMD) owns ROWS query rows and
// walks the words in windows of W; the query words and the class operand of
// a window go from global memory straight into an LDS ring of NST stages
// (global_load_lds, 16 bytes per lane), NST - 1 windows ahead of the
// window being multiplied, with one barrier per window; several workgroups
// share each CU.
#include <limits.h>

#include "hdc_stream.h"

namespace hdc {

struct HamLayout {
    int w_lo, w_hi, nwin, KT;
    size_t off_popc, total;
    HamLayout(int start, int end, int K)
    {
        w_lo = (start >> 6) & ~1;
        w_hi = (end + 63) >> 6;
        nwin = (w_hi - w_lo + kHmWin - 1) / kHmWin;
        KT = class_tiles(K);
        const size_t tab = (size_t)nwin * kHmWin * KT * 1024;
        off_popc = tab;
        total = off_popc + 128 * 4;
    }
};

size_t ham_workspace_bytes(int start, int end, int K) { return HamLayout(start, end, K).total; }

template <int KT>
__global__ __launch_bounds__(256) void k_hamming_mfma(const uint64_t *__restrict__ Q, int64_t n, int64_t ldq, int K,
                                                      int w_lo, int w_hi, int nwin, const int8_t *__restrict__ tab,
                                                      const int32_t *__restrict__ popc, int32_t *__restrict__ argmin,
                                                      int32_t *__restrict__ min_dist, int32_t *__restrict__ dists)
{
    typedef HmShape<KT> S;
    constexpr int QT = S::QT, W = S::W, ROWS = S::ROWS, NST = S::NST;
    __shared__ __align__(16) uint8_t smem[NST * S::SB];
    lds_u8 *L = (lds_u8 *)smem;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 5;
    const int64_t rbase = (int64_t)blockIdx.x * ROWS;
    const uint64_t *Qwg = Q + rbase * ldq;   // this workgroup's rows

    // Per-lane sources of the query loads: load i of a wave fills stage
    // bytes [(i * 4 + wave) * 1024, +1024) = rows RPL*j .. RPL*j + RPL-1
    // (j = i * 4 + wave), lane l -> row RPL*j + l/U, slot l%U, which holds
    // unit hm_slot(row, l%U) of the window.  Rows past n re-read row n-1.
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
    // loads of window v (clamped to the last) into stage st
    auto issue = [&](int v, int st) {
        const int vc = v < nwin ? v : nwin - 1;
        lds_u8 *sq = L + st * S::SB;
#pragma unroll
        for (int i = 0; i < S::NQL; ++i) {
            // words past the hypervector re-read the first pair (class bytes are 0 there)
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
    constexpr int G = S::NQL + S::NTL;   // loads per wave per window

    v16f acc[KT][QT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int qt = 0; qt < QT; ++qt)
            acc[kt][qt] = v16f{};

#pragma unroll
    for (int v = 0; v < NST - 1; ++v)
        issue(v, v);
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(G * (NST - 2)) : "memory");

    int st = 0;
    for (int v = 0; v < nwin; ++v) {
        issue(v + NST - 1, st == 0 ? NST - 1 : st - 1);
        const lds_u8 *sq = L + st * S::SB;
        const lds_u8 *stb = sq + S::QB;
        // query words of this wave's tiles: U 16-byte units per row
        v4i qv[QT][S::U];
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            const int r = (wave * QT + qt) * 32 + (lane & 31);
#pragma unroll
            for (int hh = 0; hh < S::U; ++hh)
                qv[qt][hh] = *(const lds_v4i *)(sq + r * (W * 8) + 16 * hm_slot<KT>(r, hh));
        }
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            v8i af[KT];
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                const v4i a4 = *(const lds_v4i *)(stb + ((ww * KT + kt) * 64 + lane) * 16);
                af[kt] = v8i{a4[0], a4[1], a4[2], a4[3], 0, 0, 0, 0};
            }
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) {
                const v4i u = qv[qt][ww >> 1];
                const uint32_t d = (uint32_t)(g ? u[2 * (ww & 1) + 1] : u[2 * (ww & 1)]);
                const v8i bf = query_nibbles(d);
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
                    acc[kt][qt] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[kt], bf, acc[kt][qt], 4, 4, 0,
                                                                                 0, 0, 0);
            }
        }
        // window v+1 complete for this wave (only the window just issued may
        // still be in flight), LDS reads done, all waves here
        asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(G * (NST - 2)) : "memory");
        st = st == NST - 1 ? 0 : st + 1;
    }
    // no load may still be writing this workgroup's LDS when it exits
    __builtin_amdgcn_s_waitcnt(0);

    // argmin: lane holds query l%32 of each tile and classes 8(v/4)+4g+v%4
#pragma unroll
    for (int qt = 0; qt < QT; ++qt) {
        const int64_t q = rbase + (wave * QT + qt) * 32 + (lane & 31);
        int bd = INT_MAX, bk = 0;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int k = kt * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
                if (k < K) {
                    const int d = popc[k] + (int)acc[kt][qt][v];
                    if (d < bd) { bd = d; bk = k; }
                    if (dists && q < n)
                        dists[q * K + k] = d;
                }
            }
        const int od = __shfl_xor(bd, 32), ok = __shfl_xor(bk, 32);
        if (od < bd || (od == bd && ok < bk)) { bd = od; bk = ok; }
        if (g == 0 && q < n) {
            argmin[q] = bk;
            if (min_dist)
                min_dist[q] = bd;
        }
    }
}

hipError_t launch_ham_prepare(const uint64_t *C, int K, int64_t ldc, int start, int end, int stride, uint8_t *ws,
                              hipStream_t st)
{
    const HamLayout L(start, end, K);
    const int64_t total = (int64_t)L.nwin * kHmWin * L.KT * 64;
    // E2M1 +2.0 / -2.0
    hipLaunchKernelGGL((k_sign_table<0x4u, 0xCu>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, C, K,
                       ldc, start, end, stride, L.w_lo, L.KT, total, (int8_t *)ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int nd = (end - start + stride - 1) / stride;
    return launch_class_popc(C, K, ldc, start, stride, nd, L.KT, (int32_t *)(ws + L.off_popc), st);
}

hipError_t launch_ham_prepared(const uint64_t *Q, int64_t n, int64_t ldq, int K, int start, int end,
                               const uint8_t *ws, int32_t *argmin, int32_t *min_dist, int32_t *dists,
                               hipStream_t st)
{
    const HamLayout L(start, end, K);
    const int8_t *tab = (const int8_t *)ws;
    const int32_t *popc = (const int32_t *)(ws + L.off_popc);
#define HDC_HM_CASE(KT_)                                                                                       \
    if (L.KT == KT_) {                                                                                         \
        constexpr int R = HmShape<KT_>::ROWS, NW = kHmWin / HmShape<KT_>::W;                                   \
        hipLaunchKernelGGL(k_hamming_mfma<KT_>, dim3((unsigned)((n + R - 1) / R)), dim3(256), 0, st, Q, n, ldq, \
                           K, L.w_lo, L.w_hi, L.nwin * NW, tab, popc, argmin, min_dist, dists);                \
        return hipGetLastError();                                                                              \
    }
    HDC_HM_CASE(1)
    HDC_HM_CASE(2)
    HDC_HM_CASE(4)
#undef HDC_HM_CASE
    return hipErrorInvalidValue;
}

}  // namespace hdc
