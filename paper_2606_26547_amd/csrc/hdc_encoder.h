// The gfx950 random-projection encoder: one 256-thread workgroup = 4
// waves, each wave owning QT tiles of 32 queries whose features stay in
// VGPRs (converted once to the compute type) for the whole launch.  The
// workgroup walks the selected dimensions 32 at a time: the 32 gathered
// projection rows of the next chunk are prefetched into registers, converted
// and written to one half of a double-buffered LDS area while the current
// chunk is multiplied on the matrix cores (rows = dimensions, columns =
// queries).  The 32x32 accumulator of each query tile then goes through one
// of two epilogues:
//   M_ENCODE   sign -> packed bits, one uint32 half-word per query per chunk
//   M_CLASSIFY sign -> {0,-1} bytes laid out as the B operand of a second
//              int8 MFMA against the +-1 class bytes of the same 32
//              dimensions (staged in LDS with the chunk), accumulating
//              sum_d c_kd * m_qd; after the last chunk the Hamming distance
//              is popc_k - acc and the argmin is taken across the lanes.
// The encoder body is a device function so the persistent configuration
// sweep can run it per work item.
#pragma once

#include "hdc_device.h"

namespace hdc {

template <int CT, int XF, int QT, int KS, int KT, int MODE>
struct Encoder {
    typedef Tr<CT> T;
    typedef typename T::frag frag;
    typedef typename T::acc acc_t;
    static constexpr int KSTEP = T::KSTEP;
    static constexpr int KB = KSTEP * T::ESZ;              // LDS bytes per K-step per row
    static constexpr int RSB = KS * KB + 16;               // LDS row stride (16 B skew)
    static constexpr int PIECES = (KS * KSTEP + 15) / 16;  // 16-byte int8 pieces per row (max)
    static constexpr int MP = (PIECES + 7) / 8;            // pieces per thread (8 threads / row)
    static constexpr int OFF_C = 2 * kDimChunk * RSB;
    static constexpr int OFF_CS = OFF_C + (MODE == M_CLASSIFY ? 2 * KT * 1024 : 0);
    static constexpr int LDS = OFF_CS + 2 * kDimChunk * 4;
    static constexpr int QPW = QT * 32;                    // queries per wave
    static constexpr int QPB = QPW * kWaves;               // queries per workgroup

    // ---------------------------------------------------------------- X
    static __device__ __forceinline__ frag load_frag(const EncodeArgs &a, int64_t q, int s, int g)
    {
        const int k0 = s * KSTEP + g * (KSTEP / 2);
        if constexpr (XF == 0) {
            const uint8_t *row = (const uint8_t *)a.X + q * a.ldx;
            const bool sgn = a.x_type == X_INT8;
            if constexpr (CT == C_I8) {
                uint4 w = *(const uint4 *)(row + k0);
                uint32_t d[4] = {w.x, w.y, w.z, w.w};
                v4i r;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t x = sgn ? d[e] : (d[e] ^ 0x80808080u);   // uint8: x - 128
                    r[e] = (int)keep_bytes(x, k0 + 4 * e, a.F);
                }
                return r;
            } else if constexpr (CT == C_FP8) {
                uint4 w0 = *(const uint4 *)(row + k0);
                uint4 w1 = *(const uint4 *)(row + k0 + 16);
                uint32_t d[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
                v8i r;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    uint32_t x = keep_bytes(d[e], k0 + 4 * e, a.F);
                    r[e] = (int)fp8x4(byte_value(x, 0, sgn), byte_value(x, 1, sgn),
                                      byte_value(x, 2, sgn), byte_value(x, 3, sgn));
                }
                return r;
            } else {   // C_BF16
                uint2 w = *(const uint2 *)(row + k0);
                uint32_t d[2] = {keep_bytes(w.x, k0, a.F), keep_bytes(w.y, k0 + 4, a.F)};
                v4i r;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    r[2 * e] = (int)bf16x2(byte_value(d[e], 0, sgn), byte_value(d[e], 1, sgn));
                    r[2 * e + 1] = (int)bf16x2(byte_value(d[e], 2, sgn), byte_value(d[e], 3, sgn));
                }
                return r;
            }
        } else {
            const float *row = (const float *)a.X + q * a.ldx;
            auto val = [&](int k) { return k < a.F ? row[k] : 0.0f; };
            if constexpr (CT == C_F32) {
                return val(k0);
            } else if constexpr (CT == C_FP8) {
                v8i r;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    float4 f = *(const float4 *)(row + k0 + 4 * e);
                    int k = k0 + 4 * e;
                    r[e] = (int)fp8x4(k < a.F ? f.x : 0.f, k + 1 < a.F ? f.y : 0.f,
                                      k + 2 < a.F ? f.z : 0.f, k + 3 < a.F ? f.w : 0.f);
                }
                return r;
            } else {   // C_BF16
                v4i r;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    float4 f = *(const float4 *)(row + k0 + 4 * e);
                    int k = k0 + 4 * e;
                    r[2 * e] = (int)bf16x2(k < a.F ? f.x : 0.f, k + 1 < a.F ? f.y : 0.f);
                    r[2 * e + 1] = (int)bf16x2(k + 2 < a.F ? f.z : 0.f, k + 3 < a.F ? f.w : 0.f);
                }
                (void)val;
                return r;
            }
        }
    }

    static __device__ __forceinline__ void load_x(frag (&xr)[QT][KS], const EncodeArgs &a,
                                                  int64_t qbase, int lane, int ks_used)
    {
        const int g = lane >> 5;
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            const int64_t q = qbase + qt * 32 + (lane & 31);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (q < a.n && s < ks_used)
                    xr[qt][s] = load_frag(a, q, s, g);
                else
                    xr[qt][s] = frag{};
            }
        }
    }

    // ---------------------------------------------------------------- P
    // Thread t stages row t/8 of the chunk, pieces t%8 + 8m.
    static __device__ __forceinline__ void stage_load(uint4 (&pr)[MP], const EncodeArgs &a, int c,
                                                      int t, int npc)
    {
        const int r = t >> 3, sub = t & 7;
        const int dl = c * kDimChunk + r;
        const bool valid = dl < a.nd;
        const int8_t *rowp = a.P + (int64_t)(a.s0 + (int64_t)dl * a.stride) * a.ldp;
#pragma unroll
        for (int m = 0; m < MP; ++m) {
            const int j = sub + 8 * m;
            if (valid && j < npc)
                pr[m] = *(const uint4 *)(rowp + 16 * j);
            else
                pr[m] = make_uint4(0, 0, 0, 0);
        }
    }

    static __device__ __forceinline__ void stage_store(uint8_t *lp, int *lcs, const uint4 (&pr)[MP],
                                                       const EncodeArgs &a, int c, int t, int npc,
                                                       bool colsum)
    {
        const int r = t >> 3, sub = t & 7;
        const bool valid = c * kDimChunk + r < a.nd;
        uint8_t *rowl = lp + r * RSB;
        int cs = 0;
#pragma unroll
        for (int m = 0; m < MP; ++m) {
            const int j = sub + 8 * m;
            if (j >= npc)
                continue;
            uint32_t d[4] = {pr[m].x, pr[m].y, pr[m].z, pr[m].w};
            if (colsum) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // sum of the +-1 weights of features < F in this dword
                    int k0 = 16 * j + 4 * e;
                    int nv = a.F - k0;
                    nv = nv < 0 ? 0 : (nv > 4 ? 4 : nv);
                    uint32_t neg = d[e] & 0x80808080u & (nv >= 4 ? 0xffffffffu : ((1u << (8 * nv)) - 1u));
                    cs += valid ? nv - 2 * __popc(neg) : 0;
                }
            }
            if constexpr (CT == C_I8) {
                *(uint4 *)(rowl + 16 * j) = pr[m];
            } else if constexpr (CT == C_FP8) {
                uint4 o;
                uint32_t *op = (uint32_t *)&o;
#pragma unroll
                for (int e = 0; e < 4; ++e)   // +1 -> 0x38, -1 -> 0xB8 (E4M3)
                    op[e] = valid ? ((d[e] & 0x80808080u) | 0x38383838u) : 0u;
                *(uint4 *)(rowl + 16 * j) = o;
            } else if constexpr (CT == C_BF16) {
                // 16 weights -> 16 bf16: +1 -> 0x3F80, -1 -> 0xBF80
                uint32_t o[8];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t sg = d[e] & 0x80808080u;
                    o[2 * e] = valid ? (0x3F803F80u | ((sg & 0x80u) << 8) | ((sg & 0x8000u) << 16)) : 0u;
                    o[2 * e + 1] = valid ? (0x3F803F80u | ((sg >> 8) & 0x8000u) | (sg & 0x80000000u)) : 0u;
                }
                *(uint4 *)(rowl + 32 * j) = make_uint4(o[0], o[1], o[2], o[3]);
                *(uint4 *)(rowl + 32 * j + 16) = make_uint4(o[4], o[5], o[6], o[7]);
            } else {   // C_F32
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t s = d[e] & 0x80808080u;
                    uint4 o = valid ? make_uint4(0x3F800000u | ((s & 0x80u) << 24), 0x3F800000u | ((s & 0x8000u) << 16),
                                                 0x3F800000u | ((s & 0x800000u) << 8), 0x3F800000u | (s & 0x80000000u))
                                    : make_uint4(0, 0, 0, 0);
                    *(uint4 *)(rowl + 64 * j + 16 * e) = o;
                }
            }
        }
        if (colsum) {
            cs += __shfl_xor(cs, 1);
            cs += __shfl_xor(cs, 2);
            cs += __shfl_xor(cs, 4);
            if (sub == 0)
                lcs[r] = cs;
        }
    }

    // ------------------------------------------------------------ classes
    static __device__ __forceinline__ uint4 class_load(const EncodeArgs &a, int c, int t)
    {
        if (t < KT * 64)
            return *(const uint4 *)(a.ctab + ((int64_t)c * KT * 64 + t) * 16);
        return make_uint4(0, 0, 0, 0);
    }
    static __device__ __forceinline__ void class_store(uint8_t *lc, uint4 v, int t)
    {
        if (t < KT * 64)
            *(uint4 *)(lc + t * 16) = v;
    }

    // ------------------------------------------------------------ compute
    static __device__ __forceinline__ void chunk_mma(acc_t (&acc)[QT], const frag (&xr)[QT][KS],
                                                     const uint8_t *lp, int lane, int ks_used)
    {
        const int g = lane >> 5, row = lane & 31;
#pragma unroll
        for (int qt = 0; qt < QT; ++qt)
            acc[qt] = acc_t{};
        const uint8_t *base = lp + row * RSB + g * (KB / 2);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s < ks_used) {
                frag af = *(const frag *)(base + s * KB);
#pragma unroll
                for (int qt = 0; qt < QT; ++qt)
                    mma(acc[qt], af, xr[qt][s]);
            }
        }
    }

    // Sign words of one tile, with the uint8 column-sum correction.
    static __device__ __forceinline__ void signs(uint32_t (&w)[16], const acc_t &acc, const int *lcs,
                                                 bool colsum, int g)
    {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            if constexpr (CT == C_I8) {
                int y = acc[v];
                if (colsum)
                    y += 128 * lcs[8 * (v >> 2) + 4 * g + (v & 3)];
                w[v] = sign_word(y);
            } else {
                w[v] = sign_word(acc[v]);
            }
        }
    }

    // ------------------------------------------------------------ body
    // Runs the whole dimension loop for the queries of this workgroup.
    // Returns the class accumulators (classify mode) through dacc.
    static __device__ __forceinline__ void run(const EncodeArgs &a, uint8_t *smem, int64_t qblock,
                                               v16i (&dacc)[KT][QT])
    {
        const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 5;
        const int64_t qbase = qblock + (int64_t)wave * QPW;
        const int ks_used = (a.F + KSTEP - 1) / KSTEP;
        const int npc = (ks_used * KSTEP + 15) / 16;
        const int NC = (a.nd + kDimChunk - 1) / kDimChunk;
        const bool colsum = CT == C_I8 && XF == 0 && a.x_type == X_UINT8;

        frag xr[QT][KS];
        load_x(xr, a, qbase, lane, ks_used);
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int qt = 0; qt < QT; ++qt)
                dacc[kt][qt] = v16i{};

        uint8_t *lp[2] = {smem, smem + kDimChunk * RSB};
        uint8_t *lc[2] = {smem + OFF_C, smem + OFF_C + KT * 1024};
        int *lcs[2] = {(int *)(smem + OFF_CS), (int *)(smem + OFF_CS) + kDimChunk};

        uint4 pr[MP];
        uint4 cr = make_uint4(0, 0, 0, 0);
        stage_load(pr, a, 0, t, npc);
        if constexpr (MODE == M_CLASSIFY)
            cr = class_load(a, 0, t);
        stage_store(lp[0], lcs[0], pr, a, 0, t, npc, colsum);
        if constexpr (MODE == M_CLASSIFY)
            class_store(lc[0], cr, t);
        __syncthreads();

        for (int c = 0; c < NC; ++c) {
            const int b = c & 1;
            const bool more = c + 1 < NC;
            if (more) {
                stage_load(pr, a, c + 1, t, npc);
                if constexpr (MODE == M_CLASSIFY)
                    cr = class_load(a, c + 1, t);
            }
            acc_t acc[QT];
            chunk_mma(acc, xr, lp[b], lane, ks_used);
            if constexpr (MODE == M_ENCODE) {
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) {
                    uint32_t w[16];
                    signs(w, acc[qt], lcs[b], colsum, g);
                    uint32_t bits = 0;
#pragma unroll
                    for (int v = 0; v < 16; ++v)
                        bits |= (w[v] >> 31) << (8 * (v >> 2) + (v & 3));
                    bits <<= 4 * g;
                    bits |= (uint32_t)__shfl_xor((int)bits, 32);
                    const int64_t q = qbase + qt * 32 + (lane & 31);
                    if (g == 0 && q < a.n)
                        a.H32[q * a.ldh32 + c] = bits;
                }
            } else {
                v4i cf[KT];
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
                    cf[kt] = *(const v4i *)(lc[b] + (kt * 64 + lane) * 16);
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) {
                    uint32_t w[16];
                    signs(w, acc[qt], lcs[b], colsum, g);
                    v4i mb;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        // bytes: 0xFF where the projection is negative, else 0
                        uint32_t t0 = __builtin_amdgcn_perm(w[4 * e + 1], w[4 * e], 0x0C0C0B09u);
                        uint32_t t1 = __builtin_amdgcn_perm(w[4 * e + 3], w[4 * e + 2], 0x0B090C0Cu);
                        mb[e] = (int)(t0 | t1);
                    }
#pragma unroll
                    for (int kt = 0; kt < KT; ++kt)
                        mma(dacc[kt][qt], cf[kt], mb);
                }
            }
            if (more) {
                stage_store(lp[b ^ 1], lcs[b ^ 1], pr, a, c + 1, t, npc, colsum);
                if constexpr (MODE == M_CLASSIFY)
                    class_store(lc[b ^ 1], cr, t);
            }
            __syncthreads();
        }
        if constexpr (MODE == M_ENCODE) {
            if (NC & 1) {   // high half of the last word holds no dimension
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) {
                    const int64_t q = qbase + qt * 32 + (lane & 31);
                    if (g == 0 && q < a.n)
                        a.H32[q * a.ldh32 + NC] = 0u;
                }
            }
        }
    }

    // Argmin over the class accumulators; returns the label of this lane's
    // query (valid in lanes 0..31 of each tile) and optionally writes dists.
    static __device__ __forceinline__ void finish(const EncodeArgs &a, int64_t qblock,
                                                  const v16i (&dacc)[KT][QT], int32_t (&lab)[QT])
    {
        const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 5;
        const int64_t qbase = qblock + (int64_t)wave * QPW;
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            const int64_t q = qbase + qt * 32 + (lane & 31);
            int bd = 0x7fffffff, bk = 0;
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int k = kt * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
                    if (k < a.K) {
                        const int d = a.cpop[k] - dacc[kt][qt][v];
                        if (d < bd) { bd = d; bk = k; }
                        if (a.dists && q < a.n)
                            a.dists[q * a.K + k] = d;
                    }
                }
            const int od = __shfl_xor(bd, 32), ok = __shfl_xor(bk, 32);
            if (od < bd || (od == bd && ok < bk)) { bd = od; bk = ok; }
            lab[qt] = bk;
        }
    }
};

}  // namespace hdc
