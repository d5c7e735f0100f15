// Device-side building blocks of the gfx950 encoder: MFMA operand traits,
// feature / weight conversion to the compute type, and the per-chunk
// sign epilogues.  Included by the HIP sources only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hdc_internal.h"

namespace hdc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// LDS (address space 3) pointer types: keeping the address space explicit
// makes the compiler emit ds_read / ds_write instead of flat accesses.
#define HDC_LDS __attribute__((address_space(3)))
typedef HDC_LDS uint8_t lds_u8;
typedef HDC_LDS int32_t lds_i32;
typedef HDC_LDS uint4 lds_uint4;
typedef HDC_LDS v4i lds_v4i;

__device__ __forceinline__ void lds_st16(lds_u8 *p, uint4 v)
{
    *(lds_v4i *)p = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
}

// Direct global -> LDS load of 16 bytes per lane: lane l's bytes at
// base + voff land at LDS address dst + 16 * l (base and dst are
// wave-uniform; they are read from the first lane, which keeps them in
// scalar registers also where the compiler cannot prove it, e.g. in a
// function that is not inlined).  Issued as inline assembly: the compiler
// then keeps counting only its own LDS reads (it would otherwise drain
// every LDS read before each MFMA), and the caller waits for these loads
// explicitly (vmcnt).
__device__ __forceinline__ void lds_dma16(const void *base, uint32_t voff, const lds_u8 *dst)
{
    const uint32_t m = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)dst);
    const uint64_t b = (uint64_t)(uintptr_t)base;
    // the builtin returns int: widen each half through uint32_t (a sign
    // extension of the low half would corrupt the high one)
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    const uint64_t bs = ((uint64_t)hi << 32) | (uint64_t)lo;
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2" ::"s"(m), "v"(voff), "s"(bs)
                 : "memory", "m0");
}

// ---------------------------------------------------------------------------
// Operand traits.  Every compute type uses a 32x32 MFMA (rows = dimensions,
// columns = queries).  KSTEP features are consumed per instruction; each
// lane supplies DW dwords of one row (A: projection row, B: query row)
// covering features [s*KSTEP + g*KSTEP/2, +KSTEP/2) with g = lane / 32.
// Accumulator lane l, register v holds row 8*(v/4) + 4*(l/32) + v%4 of
// column l % 32.
// ---------------------------------------------------------------------------
template <int CT> struct Tr;
// frag is the A operand (projection rows, from LDS), xfrag the B operand
// (query features, kept in registers); they differ for the split E4M3
// type, whose B operand is a pair: the high parts in elements 0..7 and the
// low parts in 8..15.
template <> struct Tr<C_I8> {
    static constexpr int KSTEP = 32, DW = 4, ESZ = 1;
    typedef v4i frag;
    typedef v4i xfrag;
    typedef v16i acc;
};
template <> struct Tr<C_FP8> {
    static constexpr int KSTEP = 64, DW = 8, ESZ = 1;
    typedef v8i frag;
    typedef v8i xfrag;
    typedef v16f acc;
};
template <> struct Tr<C_FP8S> {
    static constexpr int KSTEP = 64, DW = 8, ESZ = 1;
    typedef v8i frag;
    typedef v16i xfrag;
    typedef v16f acc;
};
template <> struct Tr<C_BF16> {
    static constexpr int KSTEP = 16, DW = 4, ESZ = 2;
    typedef v4i frag;           // 8 bf16 reinterpreted
    typedef v4i xfrag;
    typedef v16f acc;
};
template <> struct Tr<C_F32> {
    static constexpr int KSTEP = 2, DW = 1, ESZ = 4;
    typedef float frag;
    typedef float xfrag;
    typedef v16f acc;
};

// Halves of a split E4M3 B operand.
__device__ __forceinline__ v8i split_hi(const v16i &x) { return __builtin_shufflevector(x, x, 0, 1, 2, 3, 4, 5, 6, 7); }
__device__ __forceinline__ v8i split_lo(const v16i &x)
{
    return __builtin_shufflevector(x, x, 8, 9, 10, 11, 12, 13, 14, 15);
}

__device__ __forceinline__ void mma(v16i &c, const v4i &a, const v4i &b)
{
    c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mma(v16f &c, const v8i &a, const v8i &b)
{
    // A and B both OCP E4M3 (format code 0), no block scaling
    c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}
__device__ __forceinline__ void mma(v16f &c, const v4i &a, const v4i &b)
{
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
__device__ __forceinline__ void mma(v16f &c, const float &a, const float &b)
{
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Sign word of an accumulator element: bit 31 set iff the projection is
// negative.  Adding +0.0 turns a -0.0 float sum into +0.0 so that an exact
// zero counts as +1 in both arithmetics.
__device__ __forceinline__ uint32_t sign_word(int y) { return (uint32_t)y; }
__device__ __forceinline__ uint32_t sign_word(float y) { return __float_as_uint(y + 0.0f); }

// ---------------------------------------------------------------------------
// Conversions to the compute type.
// ---------------------------------------------------------------------------
// Four floats -> four OCP E4M3 bytes (round to nearest even), saturating at
// +-448 like the format's "satfinite" conversion.
__device__ __forceinline__ uint32_t fp8x4(float a, float b, float c, float d)
{
    a = fminf(fmaxf(a, -448.f), 448.f);
    b = fminf(fmaxf(b, -448.f), 448.f);
    c = fminf(fmaxf(c, -448.f), 448.f);
    d = fminf(fmaxf(d, -448.f), 448.f);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
}

// Two floats -> two bfloat16 (round to nearest even) packed low/high.
__device__ __forceinline__ uint32_t bf16x2(float a, float b)
{
    typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
    v2bf r = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, r);
}

// Byte e of a dword as a float, for signed or unsigned 8-bit features.
__device__ __forceinline__ float byte_value(uint32_t w, int e, bool is_signed)
{
    uint32_t b = (w >> (8 * e)) & 0xffu;
    return is_signed ? (float)(int)(int8_t)b : (float)b;
}

// Four integer features (bytes of w, signed or unsigned) split into E4M3
// parts: *hi gets 16 * floor(x / 16) (the byte with its low nibble cleared,
// read with the feature's sign: a multiple of 16 in [-128, 240]), *lo gets
// x mod 16 (the low nibble, 0..15).  Both are exact in E4M3 (four
// significant bits), so the conversions do not round.
__device__ __forceinline__ void fp8_split4(uint32_t w, bool is_signed, uint32_t *hi, uint32_t *lo)
{
    const uint32_t h = w & 0xF0F0F0F0u, l = w & 0x0F0F0F0Fu;
    *hi = fp8x4(byte_value(h, 0, is_signed), byte_value(h, 1, is_signed), byte_value(h, 2, is_signed),
                byte_value(h, 3, is_signed));
    *lo = fp8x4((float)(l & 0xffu), (float)((l >> 8) & 0xffu), (float)((l >> 16) & 0xffu), (float)(l >> 24));
}

// Keep the bytes of w whose feature index (k0 + byte) is below F.
__device__ __forceinline__ uint32_t keep_bytes(uint32_t w, int k0, int F)
{
    int v = F - k0;
    if (v >= 4) return w;
    if (v <= 0) return 0u;
    return w & ((1u << (8 * v)) - 1u);
}

}  // namespace hdc
