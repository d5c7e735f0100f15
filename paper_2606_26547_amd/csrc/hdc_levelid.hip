// Encode-side kernels beside random projection: the feature-column gather
// that perforates the encoding's reduction over features, the level
// quantiser and Level-ID encoding.
//
// Level-ID: bit d of a row's hypervector is set when more than half of the
// F bound pairs ID_f xor LV_level(f) have bit d set (the bipolar sum is
// F - 2*count; a zero sum gives +1).  One thread owns 64 dimensions of one
// row; per feature it XORs the ID word with the level word (both from LDS;
// levels come 8 to a 16-byte load) and adds the result to a bit-sliced
// counter through a carry-save (Harley-Seal) tree: 16 inputs take 15
// three-operation adders and one ripple add of the weight-16 carries,
// about four operations per input and 32-bit half.
#include "hdc_device.h"

namespace hdc {

// ------------------------------------------------------------------ gather
// Y[i][j] = X[i][start + j*stride] for j < nf, 0 for nf <= j < ldy; each
// thread writes 16 bytes of one row.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_cols(const T *__restrict__ X, int64_t n, int64_t ldx, int start,
                                                     int stride, int nf, T *__restrict__ Y, int64_t ldy)
{
    constexpr int E = 16 / sizeof(T);
    const int64_t per_row = ldy / E;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * per_row)
        return;
    const int64_t i = idx / per_row;
    const int j0 = (int)(idx - i * per_row) * E;
    const T *x = X + i * ldx + start;
    T v[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = j0 + e < nf ? x[(int64_t)(j0 + e) * stride] : T(0);
    *(uint4 *)(Y + i * ldy + j0) = *(const uint4 *)v;
}

hipError_t launch_gather_cols(const void *X, int elem, int64_t n, int64_t ldx, int start, int stride, int nf,
                              void *Y, int64_t ldy, hipStream_t st)
{
    const int64_t total = n * (ldy * elem / 16);
    const dim3 grid((unsigned)((total + 255) / 256));
    if (elem == 1)
        hipLaunchKernelGGL(k_gather_cols<uint8_t>, grid, dim3(256), 0, st, (const uint8_t *)X, n, ldx, start,
                           stride, nf, (uint8_t *)Y, ldy);
    else
        hipLaunchKernelGGL(k_gather_cols<float>, grid, dim3(256), 0, st, (const float *)X, n, ldx, start, stride,
                           nf, (float *)Y, ldy);
    return hipGetLastError();
}

// --------------------------------------------------------------- quantiser
// level = floor((x - lo) * L / (hi - lo)) in binary32, each step rounded to
// nearest even (no contraction), 0 for an empty range, a value at or below
// lo, or NaN; L - 1 at or above the top level.
__global__ __launch_bounds__(256) void k_level_quantize(const float *__restrict__ X, int64_t n, int F, int64_t ldx,
                                                        const float *__restrict__ lo, const float *__restrict__ hi,
                                                        int L, uint16_t *__restrict__ lev, int64_t ldl)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * F)
        return;
    const int64_t i = idx / F;
    const int f = (int)(idx - i * F);
    const float t = __fsub_rn(X[i * ldx + f], lo[f]);
    const float w = __fsub_rn(hi[f], lo[f]);
    const float v = __fdiv_rn(__fmul_rn(t, (float)L), w);
    int level;
    if (!(w > 0.0f) || !(v > 0.0f))
        level = 0;
    else if (v >= (float)(L - 1))
        level = L - 1;
    else
        level = (int)floorf(v);
    lev[i * ldl + f] = (uint16_t)level;
}

hipError_t launch_level_quantize(const float *X, int64_t n, int F, int64_t ldx, const float *lo, const float *hi,
                                 int L, uint16_t *lev, int64_t ldl, hipStream_t st)
{
    const int64_t total = n * F;
    hipLaunchKernelGGL(k_level_quantize, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X, n, F, ldx, lo,
                       hi, L, lev, ldl);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Level-ID
constexpr int kLidWords = 8;    // 64-bit words (512 dimensions) per workgroup
constexpr int kLidRows = 32;    // rows per pass of a workgroup (256 threads / 8 words)
constexpr int kLidPasses = 4;   // passes over one staged window (128 rows per workgroup)
constexpr int kLidLvPitch = 9;  // padded level-row pitch in LDS (64-bit words)
constexpr int kLidBig = 7;      // planes of the weight-16 counter (F <= 1024 -> count/16 <= 64)

size_t lid_lds_bytes(int F, int L) { return ((size_t)F * kLidWords + (size_t)L * kLidLvPitch) * 8; }

// carry-save adder: (h, l) = (majority, parity) of (a, b, c)
__device__ __forceinline__ void csa(uint64_t &h, uint64_t &l, uint64_t a, uint64_t b, uint64_t c)
{
    const uint64_t u = a ^ b;
    h = ((a ^ c) & u) ^ a;      // a where a == b, c elsewhere (a bit select)
    l = u ^ c;
}

struct LidCounter {
    uint64_t ones = 0, twos = 0, fours = 0, eights = 0, big[kLidBig] = {};

    // add 16 one-bit inputs per dimension
    __device__ __forceinline__ void add16(const uint64_t (&x)[16])
    {
        uint64_t ta, tb, fa, fb, ea, eb, sixteens;
        csa(ta, ones, ones, x[0], x[1]);
        csa(tb, ones, ones, x[2], x[3]);
        csa(fa, twos, twos, ta, tb);
        csa(ta, ones, ones, x[4], x[5]);
        csa(tb, ones, ones, x[6], x[7]);
        csa(fb, twos, twos, ta, tb);
        csa(ea, fours, fours, fa, fb);
        csa(ta, ones, ones, x[8], x[9]);
        csa(tb, ones, ones, x[10], x[11]);
        csa(fa, twos, twos, ta, tb);
        csa(ta, ones, ones, x[12], x[13]);
        csa(tb, ones, ones, x[14], x[15]);
        csa(fb, twos, twos, ta, tb);
        csa(eb, fours, fours, fa, fb);
        csa(sixteens, eights, eights, ea, eb);
        uint64_t c = sixteens;
#pragma unroll
        for (int p = 0; p < kLidBig; ++p) {
            const uint64_t nc = big[p] & c;
            big[p] ^= c;
            c = nc;
        }
    }

    // count = ones + 2 twos + 4 fours + 8 eights + 16 big: one plane per
    // weight, i.e. the count's binary digits; returns count > T per bit.
    __device__ __forceinline__ uint64_t greater(uint32_t T) const
    {
        uint64_t cnt[4 + kLidBig] = {ones, twos, fours, eights};
#pragma unroll
        for (int p = 0; p < kLidBig; ++p)
            cnt[4 + p] = big[p];
        uint64_t gt = 0, eq = ~0ull;
#pragma unroll
        for (int p = 4 + kLidBig - 1; p >= 0; --p) {
            if ((T >> p) & 1u) {
                eq &= cnt[p];
            } else {
                gt |= eq & cnt[p];
                eq &= ~cnt[p];
            }
        }
        return gt;
    }
};

// Bit word of one row: dimensions of the thread's word where more than half
// of the F bound pairs are -1.
__device__ __forceinline__ uint64_t level_id_word(const uint16_t *__restrict__ lrow, int F, int L,
                                                  const HDC_LDS uint64_t *sidw, const HDC_LDS uint64_t *slvw)
{
    const uint4 *lr = (const uint4 *)lrow;                 // 8 levels per 16 bytes
    LidCounter cnt;
    const int Ffull = F & ~15;
    int f0 = 0;
    for (; f0 < Ffull; f0 += 16) {
        const uint4 a = lr[f0 / 8], b = lr[f0 / 8 + 1];
        const uint32_t lw[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint64_t x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint32_t l = min((lw[u / 2] >> (16 * (u & 1))) & 0xffffu, (uint32_t)L - 1u);
            x[u] = sidw[(f0 + u) * kLidWords] ^ slvw[__umul24(l, (uint32_t)kLidLvPitch)];
        }
        cnt.add16(x);
    }
    if (f0 < F) {                                      // tail: F - f0 < 16 features
        uint64_t x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            x[u] = 0;
            if (f0 + u < F) {
                const int l = min((int)lrow[f0 + u], L - 1);
                x[u] = sidw[(f0 + u) * kLidWords] ^ slvw[l * kLidLvPitch];
            }
        }
        cnt.add16(x);
    }
    return cnt.greater((uint32_t)F >> 1);
}

__global__ __launch_bounds__(256) void k_level_id(const uint16_t *__restrict__ lev, int64_t n, int F, int64_t ldl,
                                                  const uint64_t *__restrict__ ID, int64_t ldid,
                                                  const uint64_t *__restrict__ LV, int L, int64_t ldlv, int D,
                                                  uint64_t *__restrict__ H, int64_t ldh)
{
    extern __shared__ __align__(16) uint64_t lds_raw[];
    typedef HDC_LDS uint64_t lds_u64;
    lds_u64 *sid = (lds_u64 *)lds_raw;                 // [F][kLidWords]
    lds_u64 *slv = sid + F * kLidWords;                // [L][kLidLvPitch]
    const int t = threadIdx.x;
    const int W = (D + 63) / 64;
    const int w0 = blockIdx.x * kLidWords;
    const int nw = min(kLidWords, W - w0);
    // staging: 8 independent loads in flight per thread before their stores
    {
        const int ne = (F + L) * kLidWords;
        for (int e0 = 0; e0 < ne; e0 += 8 * 256) {
            uint64_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int e = e0 + j * 256 + t;
                const int r = e / kLidWords, w = e % kLidWords;
                v[j] = 0;
                if (e < ne && w < nw)
                    v[j] = r < F ? ID[(int64_t)r * ldid + w0 + w] : LV[(int64_t)(r - F) * ldlv + w0 + w];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int e = e0 + j * 256 + t;
                const int r = e / kLidWords, w = e % kLidWords;
                if (e < ne) {
                    if (r < F)
                        sid[e] = v[j];
                    else
                        slv[(r - F) * kLidLvPitch + w] = v[j];
                }
            }
        }
    }
    __syncthreads();

    const int wi = t % kLidWords;
    if (wi >= nw)
        return;
    const lds_u64 *sidw = sid + wi;
    const lds_u64 *slvw = slv + wi;
    const int wg = w0 + wi;
    const uint64_t tail_mask = (wg == W - 1 && (D & 63)) ? (1ull << (D & 63)) - 1ull : ~0ull;
    for (int pass = 0; pass < kLidPasses; ++pass) {
        const int64_t row = ((int64_t)blockIdx.y * kLidPasses + pass) * kLidRows + t / kLidWords;
        if (row >= n)
            break;
        H[row * ldh + wg] = level_id_word(lev + row * ldl, F, L, sidw, slvw) & tail_mask;
    }
}

hipError_t launch_level_id(const uint16_t *lev, int64_t n, int F, int64_t ldl, const uint64_t *ID, int64_t ldid,
                           const uint64_t *LV, int L, int64_t ldlv, int D, uint64_t *H, int64_t ldh, hipStream_t st)
{
    const size_t lds = lid_lds_bytes(F, L);
    // once per process (thread-safe static initialisation)
    static const hipError_t attr = hipFuncSetAttribute((const void *)k_level_id,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess)
        return attr;
    const int W = (D + 63) / 64;
    const int64_t rows_per_wg = (int64_t)kLidRows * kLidPasses;
    const dim3 grid((unsigned)((W + kLidWords - 1) / kLidWords), (unsigned)((n + rows_per_wg - 1) / rows_per_wg));
    hipLaunchKernelGGL(k_level_id, grid, dim3(256), lds, st, lev, n, F, ldl, ID, ldid, LV, L, ldlv, D, H, ldh);
    return hipGetLastError();
}

}  // namespace hdc
