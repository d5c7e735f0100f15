// Shared skeleton of the prepared bit-vector searches (Hamming, ADC): the
// shape of a workgroup's LDS ring and the FP4 query operand.
#pragma once

#include "hdc_device.h"

namespace hdc {

// Shape per class-tile count: query tiles (32 queries) per wave, words per
// window, LDS stages.  Two stages keep the LDS footprint small enough for
// several workgroups per CU: the other waves on each SIMD cover one wave's
// operand building, LDS waits and barriers, which pays more than deeper
// prefetch.
template <int KT> struct HmShape {
    static constexpr int QT = KT == 4 ? 1 : 2;
    static constexpr int W = KT == 1 ? 8 : 4;          // words per window (divides kHmWin)
    static constexpr int U = W / 2;                    // 16-byte units per query row
    static constexpr int RPL = 64 / U;                 // query rows per 1 KiB load
    static constexpr int SWZ = U == 2 ? 3 : 2;         // row shift of the unit swizzle
    static constexpr int ROWS = kWaves * QT * 32;      // queries per workgroup
    static constexpr int QB = ROWS * W * 8;            // query bytes per stage
    static constexpr int TB = W * KT * 1024;           // class operand bytes per window
    static constexpr int NST = 2;                      // LDS stages
    static constexpr int NQL = QB / 1024 / kWaves;     // query loads per wave per window
    static constexpr int NTL = TB / 1024 / kWaves;     // class loads per wave per window
    static constexpr int SB = QB + TB;                 // bytes per stage
};
constexpr int kHmWin = 8;   // the class operand is padded to whole 8-word windows

// Query bits of one dword as the FP4 B operand (0.5 per set bit): register
// r, nibble j = bit 4j + r.  The upper half of the operand is unused by FP4.
__device__ __forceinline__ v8i query_nibbles(uint32_t d)
{
    v8i b = {};
#pragma unroll
    for (int r = 0; r < 4; ++r)
        b[r] = (int)((d >> r) & 0x11111111u);
    return b;
}

// Query bits of one dword as bipolar FP4 values: +1.0 (0x2) for a clear bit,
// -1.0 (0xA) for a set one, in the same nibble order as query_nibbles.
__device__ __forceinline__ v8i query_bipolar(uint32_t d)
{
    v8i b = {};
#pragma unroll
    for (int r = 0; r < 4; ++r)
        b[r] = (int)((((d >> r) & 0x11111111u) << 3) | 0x22222222u);
    return b;
}

// Class operand table of the FP4 searches: for word w (from w_lo) and class
// tile kt, 64 lanes x 16 bytes where lane l, nibble j of dword r holds, for
// class kt*32 + l%32 at dimension d = 64w + 32*(l/32) + 4j + r, the code
// POS (class bit 0) or NEG (class bit 1) when d is in S, else 0.
template <uint32_t POS, uint32_t NEG>
__global__ __launch_bounds__(256) void k_sign_table(const uint64_t *__restrict__ C, int K, int64_t ldc, int start,
                                                    int end, int stride, int w_lo, int KT, int64_t total,
                                                    int8_t *__restrict__ tab)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total)
        return;
    const int lane = (int)(idx & 63);
    const int kt = (int)((idx >> 6) % KT);
    const int64_t w = w_lo + (idx >> 6) / KT;
    const int k = kt * 32 + (lane & 31), g = lane >> 5;
    uint32_t o[4] = {0, 0, 0, 0};
    if (k < K) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t d = w * 64 + 32 * g + 4 * j + r;
                if (d >= start && d < end && (d - start) % stride == 0) {
                    const int bit = (int)((C[k * ldc + (d >> 6)] >> (d & 63)) & 1u);
                    o[r] |= (bit ? NEG : POS) << (4 * j);
                }
            }
    }
    *(uint4 *)(tab + idx * 16) = make_uint4(o[0], o[1], o[2], o[3]);
}

// Query row r of a stage is W words = U 16-byte units; unit hh of the
// window sits in slot hh ^ ((r >> SWZ) & (U - 1)), which keeps the 16-byte
// reads of 16 consecutive rows on distinct banks.
template <int KT> __device__ __forceinline__ int hm_slot(int r, int hh)
{
    typedef HmShape<KT> S;
    return hh ^ ((r >> S::SWZ) & (S::U - 1));
}

}  // namespace hdc
