// The gfx950 random-projection encoder: one 256-thread workgroup = 4
// waves, each wave owning QT tiles of 32 queries whose features stay in
// VGPRs (converted once to the compute type) for the whole launch.  The
// workgroup walks the selected dimensions 32 at a time: the 32 gathered
// projection rows of the next chunk are prefetched into registers, converted
// and written to one half of a double-buffered LDS area while the current
// chunk is multiplied on the matrix cores (rows = dimensions, columns =
// queries).  The 32x32 accumulator of each query tile then goes through one
// of two epilogues, which run between the MFMAs of the following chunk:
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

template <int CT, int XF, int QT, int KS, int KT, int MODE, int WV = 0, bool DMA = false, int RT = 1>
struct Encoder {
    typedef Tr<CT> T;
    typedef typename T::frag frag;
    typedef typename T::xfrag xfrag;
    typedef typename T::acc acc_t;
    static constexpr int KSTEP = T::KSTEP;
    static constexpr int KB = KSTEP * T::ESZ;              // LDS bytes per K-step per row
    static constexpr int RSB = KS * KB + 16;               // LDS row stride (16 B skew)
    static constexpr int PIECES = (KS * KSTEP + 15) / 16;  // 16-byte int8 pieces per row (max)
    static constexpr int MP = (PIECES + 7) / 8;            // pieces per thread (8 threads / row)
    // DMA: projection rows and class fragments go from global memory
    // straight into LDS (global_load_lds, 16 bytes per lane), three stages
    // deep.  Each load fills 1 KiB of LDS contiguously, so a stage is NIW
    // loads per wave and the units past the 32 rows land in the stage's
    // slack.  The rows are copied as they are: int8 +-1 for the int8 path,
    // or the shifted weights 0 / 2 with poff set (int8 features: uint8 ones
    // would need column sums), or rows already in the compute type (bf16 /
    // E4M3 +-1.0, built once by the caller) for those paths, which take
    // either feature type.
    // A chunk is RT row tiles of 32 dimensions (RT > 1 with DMA staging
    // only; three row tiles classify only, in two stages); its class operand
    // is RT * KT KiB.
    static_assert(!DMA || (XF == 0 && (CT == C_I8 || CT == C_BF16 || CT == C_FP8)),
                  "direct LDS staging is for integer features on the int8, bf16 and E4M3 paths");
    static_assert(RT == 1 || DMA, "several row tiles per chunk need direct LDS staging");
    static_assert(RT != 3 || MODE == M_CLASSIFY, "three row tiles per chunk: classify only");
    static constexpr int CH = kDimChunk * RT;              // dimensions per chunk
    static constexpr int UPR = RSB / 16;                   // 16-byte units per LDS row
    static constexpr int NIW = (CH * UPR + 64 * kWaves - 1) / (64 * kWaves);
    static constexpr int NCT = RT * KT;                    // class tiles per chunk
    static constexpr int NCW = (NCT + kWaves - 1) / kWaves;   // class-tile loads per wave
    static constexpr int NBUF = DMA ? (RT == 3 ? 2 : 3) : 2;   // LDS stages
    static constexpr int SSZ = DMA ? NIW * kWaves * 1024 : CH * RSB;   // bytes per stage
    static constexpr int OFF_C = NBUF * SSZ;
    static constexpr int OFF_CS = OFF_C + (MODE == M_CLASSIFY ? NBUF * NCT * 1024 : 0);
    static constexpr int LDS = OFF_CS + (DMA ? 0 : NBUF * kDimChunk * 4);
    static constexpr int QPW = QT * 32;                    // queries per wave
    // Waves per SIMD the kernel is compiled for (WV, or by default two where
    // the resident query operand leaves room, so that one wave's stalls are
    // covered by the other's MFMAs, else one).
    static constexpr int WAVES = WV ? WV
                                    : ((QT == 1 && RT == 1 && KT == 1 &&
                                        ((CT == C_I8 && KS <= 20) || (CT == C_BF16 && KS <= 16) ||
                                         (CT == C_F32 && KS <= 64))) ? 2 : 1);
    static constexpr int QPB = QPW * kWaves;               // queries per workgroup

    // ---------------------------------------------------------------- X
    static __device__ __forceinline__ xfrag load_frag(const EncodeArgs &a, int64_t q, int s, int g)
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
            } else if constexpr (CT == C_FP8S) {
                uint4 w0 = *(const uint4 *)(row + k0);
                uint4 w1 = *(const uint4 *)(row + k0 + 16);
                uint32_t d[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
                v16i r;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    uint32_t hi, lo;
                    fp8_split4(keep_bytes(d[e], k0 + 4 * e, a.F), sgn, &hi, &lo);
                    r[e] = (int)hi;
                    r[8 + e] = (int)lo;
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
            static_assert(CT != C_FP8S, "the split E4M3 type is for integer features");
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

    static __device__ __forceinline__ void load_x(xfrag (&xr)[QT][KS], const EncodeArgs &a,
                                                  int64_t qbase, int lane, int ks_used)
    {
        // Branch-free: out-of-range rows / steps load an in-bounds address
        // (row n-1, step 0) and are zeroed, so all loads are in flight at once.
        const int g = lane >> 5;
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            const int64_t q = qbase + qt * 32 + (lane & 31);
            const bool qv = q < a.n;
            const int64_t qc = qv ? q : a.n - 1;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const bool v = qv && s < ks_used;
                xfrag f = load_frag(a, qc, v ? s : 0, g);
                if (!v)
                    f = xfrag{};
                xr[qt][s] = f;
            }
        }
    }

    // Start of chain 0 of each query tile on the int8 path: with the
    // shifted projection (weights p + 1 in {0, 2}, poff set) the MFMAs add
    // sum_i x_i (p_i + 1) = y + sum_i x_i, so the chain starts from minus
    // the query's feature sum and ends at y exactly (integer arithmetic);
    // otherwise from 0.  Lane l holds half of every K step of query l % 32
    // (features past F are zero in xr); the two halves are added across the
    // lane pair.  Shifted weights are mostly zero bits: the matrix cores
    // switch far fewer of them than on +-1 (0x01 / 0xFF) and hold a higher
    // clock under full load.  The E4M3 path (weights 0 / 2.0) takes minus
    // the sum of its rounded features from the matrix cores (an all -1.0
    // operand against the query fragments; integers below 2^24, exact in
    // fp32).  Only the shapes the shifted types launch take the shifted
    // projection (int8: two query tiles, shift_tile; E4M3: one query tile,
    // shift8_tile); the others start from 0.
    static constexpr bool kShift = DMA && ((CT == C_I8 && QT == 2 && shift_tile(KS, KT)) ||
                                           (CT == C_FP8 && QT == 1 && shift8_tile(KS, KT)));
    static __device__ __forceinline__ void shift_start(acc_t (&x0)[QT], const xfrag (&xr)[QT][KS], int poff)
    {
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            if constexpr (kShift && CT == C_FP8) {
                const int m1 = poff ? (int)0xB8B8B8B8u : 0;   // E4M3 -1.0 bytes, or zeros
                frag neg;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    neg[i] = m1;
                x0[qt] = acc_t{};
#pragma unroll
                for (int k = 0; k < KS; ++k)
                    mma(x0[qt], neg, xr[qt][k]);
            } else if constexpr (kShift) {
                int s = 0;
#pragma unroll
                for (int k = 0; k < KS; ++k)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        s = __builtin_amdgcn_sdot4(xr[qt][k][e], 0x01010101, s, false);
                s += __shfl_xor(s, 32);
                const int v = poff ? -s : 0;
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    x0[qt][i] = v;
            } else {
                x0[qt] = acc_t{};
            }
        }
    }

    // ---------------------------------------------------------------- P
    // Thread t stages row t/8 of the chunk, pieces t%8 + 8m.
    static __device__ __forceinline__ void stage_load(uint4 (&pr)[MP], const EncodeArgs &a, int c,
                                                      int t, int npc)
    {
        // Branch-free: rows past the dimension list re-read row S_0 and
        // pieces past the row re-read piece 0; stage_store discards both.
        const int r = t >> 3, sub = t & 7;
        const int dl = c * kDimChunk + r;
        const int dlc = dl < a.nd ? dl : 0;
        const int8_t *rowp = a.P + (int64_t)(a.s0 + (int64_t)dlc * a.stride) * a.ldp;
#pragma unroll
        for (int m = 0; m < MP; ++m) {
            const int j = sub + 8 * m;
            pr[m] = *(const uint4 *)(rowp + 16 * (j < npc ? j : 0));
        }
    }

    // Zero the part of every LDS row past the staged pieces (both buffers),
    // so that the fixed-length K loop multiplies zero features by finite
    // weights there.  Disjoint from what stage_store writes.
    static __device__ __forceinline__ void zero_tails(lds_u8 *lp0, lds_u8 *lp1, int t, int npc)
    {
        const int r = t >> 3, sub = t & 7;
        const int used16 = npc * T::ESZ, tot16 = KS * KB / 16;
        for (int u = used16 + sub; u < tot16; u += 8) {
            lds_st16(lp0 + r * RSB + 16 * u, make_uint4(0, 0, 0, 0));
            lds_st16(lp1 + r * RSB + 16 * u, make_uint4(0, 0, 0, 0));
        }
    }

    static __device__ __forceinline__ void stage_store(lds_u8 *lp, lds_i32 *lcs, const uint4 (&pr)[MP],
                                                       const EncodeArgs &a, int c, int t, int npc,
                                                       bool colsum)
    {
        const int r = t >> 3, sub = t & 7;
        const bool valid = c * kDimChunk + r < a.nd;
        lds_u8 *rowl = lp + r * RSB;
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
                lds_st16(rowl + 16 * j, valid ? pr[m] : make_uint4(0, 0, 0, 0));
            } else if constexpr (CT == C_FP8 || CT == C_FP8S) {
                uint4 o;
                uint32_t *op = (uint32_t *)&o;
#pragma unroll
                for (int e = 0; e < 4; ++e)   // +1 -> 0x38, -1 -> 0xB8 (E4M3)
                    op[e] = valid ? ((d[e] & 0x80808080u) | 0x38383838u) : 0u;
                lds_st16(rowl + 16 * j, o);
            } else if constexpr (CT == C_BF16) {
                // 16 weights -> 16 bf16: +1 -> 0x3F80, -1 -> 0xBF80
                uint32_t o[8];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t sg = d[e] & 0x80808080u;
                    o[2 * e] = valid ? (0x3F803F80u | ((sg & 0x80u) << 8) | ((sg & 0x8000u) << 16)) : 0u;
                    o[2 * e + 1] = valid ? (0x3F803F80u | ((sg >> 8) & 0x8000u) | (sg & 0x80000000u)) : 0u;
                }
                lds_st16(rowl + 32 * j, make_uint4(o[0], o[1], o[2], o[3]));
                lds_st16(rowl + 32 * j + 16, make_uint4(o[4], o[5], o[6], o[7]));
            } else {   // C_F32
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t s = d[e] & 0x80808080u;
                    uint4 o = valid ? make_uint4(0x3F800000u | ((s & 0x80u) << 24), 0x3F800000u | ((s & 0x8000u) << 16),
                                                 0x3F800000u | ((s & 0x800000u) << 8), 0x3F800000u | (s & 0x80000000u))
                                    : make_uint4(0, 0, 0, 0);
                    lds_st16(rowl + 64 * j + 16 * e, o);
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
        // threads past the table re-read entry 0 (discarded by class_store)
        const int tc = t < KT * 64 ? t : 0;
        return *(const uint4 *)(a.ctab + ((int64_t)c * KT * 64 + tc) * 16);
    }
    static __device__ __forceinline__ void class_store(lds_u8 *lc, uint4 v, int t)
    {
        if (t < KT * 64)
            lds_st16(lc + t * 16, v);
    }

    // ------------------------------------------------------------ compute
    // A dependent MFMA chain issues at half rate on gfx950 (the result
    // latency is twice the issue interval), so a single-tile wave alternates
    // its K steps between KC = 2 accumulators, added in the epilogue: exact
    // for int32, and order-free for the float rungs on integer-valued
    // features (sums below 2^24).  Register-staged kernels compiled for two
    // waves per SIMD have no room for the second set and rely on the other
    // wave instead; two query tiles are two chains already.
    // The split E4M3 type always has two: its high parts accumulate in the
    // first, its low parts in the second (|sums| < 2^24, exact).
    static constexpr int KC = CT == C_FP8S ? 2 : (QT == 1 && (WAVES == 1 || DMA) && KS >= 2) ? 2 : 1;
    typedef acc_t Parts[QT][KC];             // accumulators of one row tile
    static constexpr int kPhases = 4 * QT;   // epilogue phases (see Epilogue)

    // Work interleaved with a pass: at(s) runs after the MFMAs of K step s,
    // tail() after the loop.
    struct NoHook {
        __device__ __forceinline__ void at(int) const {}
        __device__ __forceinline__ void tail() const {}
    };

    // One pass over a row tile (32 dimensions) in LDS: a fixed-length,
    // branch-free K loop with PD projection fragments in flight (steps past
    // the feature count read zero-filled or finite LDS against zero
    // features).  Chain 0 of every query tile starts from x0 (minus the
    // query's feature sum on the shifted projection, else 0), or from the
    // uint8 correction 128 * sum_i p_i of its rows.  The hook's work (the
    // previous row tile's epilogue, the next chunk's loads) issues between
    // the MFMAs, while the matrix core is busy.
    template <class Hook>
    static __device__ __forceinline__ void tile_mma(Parts &part, const xfrag (&xr)[QT][KS], const lds_u8 *lp,
                                                    const lds_i32 *lcs, bool colsum, int lane, const Hook &hook,
                                                    const acc_t (&x0)[QT])
    {
        const int g = lane >> 5, row = lane & 31;
        const lds_u8 *base = lp + row * RSB + g * (KB / 2);
        constexpr int PDW = (CT == C_I8 && (WAVES == 1 || DMA)) ? 4 : (CT == C_F32 ? 4 : 2);
        constexpr int PD = KS < PDW ? KS : PDW;
        frag f[PD];
#pragma unroll
        for (int s = 0; s < PD; ++s)
            f[s] = *(const HDC_LDS frag *)(base + s * KB);
#pragma unroll
        for (int qt = 0; qt < QT; ++qt)
#pragma unroll
            for (int k = 0; k < KC; ++k)
                part[qt][k] = k == 0 ? x0[qt] : acc_t{};
        if constexpr (CT == C_I8) {
            if (colsum) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const v4i cs = *(const lds_v4i *)(lcs + 8 * j + 4 * g);
#pragma unroll
                    for (int qt = 0; qt < QT; ++qt)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            part[qt][0][4 * j + i] = 128 * cs[i];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const frag cur = f[s % PD];
            if (s + PD < KS)
                f[s % PD] = *(const HDC_LDS frag *)(base + (s + PD) * KB);
            if constexpr (CT == C_FP8S) {
#pragma unroll
                for (int qt = 0; qt < QT; ++qt)
                    mma(part[qt][0], cur, split_hi(xr[qt][s]));
#pragma unroll
                for (int qt = 0; qt < QT; ++qt)
                    mma(part[qt][1], cur, split_lo(xr[qt][s]));
            } else {
#pragma unroll
                for (int qt = 0; qt < QT; ++qt)
                    mma(part[qt][s % KC], cur, xr[qt][s]);
            }
            hook.at(s);
            __builtin_amdgcn_sched_barrier(0);
        }
        hook.tail();
    }

    // Epilogue of row tile w (dimensions S_{32w .. 32w+31}) split into
    // phases; per query tile qt:
    //   4qt     adds the KC partial accumulators
    //   classify: 4qt+1, 4qt+2 turn the signs into {0,-1} bytes (the B
    //             operand), 4qt+3 runs the Hamming MFMAs against the class
    //             fragments of the tile
    //   encode:   4qt+1, 4qt+2 pack the 16 signs of the lane, join the two
    //             lane halves and clear dimensions past the end, 4qt+3
    //             stores the 32-bit word
    struct Epilogue {
        const EncodeArgs &a;
        Parts &part;
        v16i (&dacc)[KT][QT];
        const v4i (&cf)[KT];
        int w, lane, g;
        int64_t qbase;
        mutable v4i mb[QT];
        mutable uint32_t bits[QT];

        __device__ __forceinline__ void operator()(int p) const
        {
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) {
                const int ph = p - 4 * qt;
                const acc_t &y = part[qt][0];
                if (ph == 0) {
                    if constexpr (CT == C_FP8 || CT == C_FP8S) {
                        // The 16-pass E4M3 MFMA's accumulator was observed to
                        // be read one wait state early by the compiler-inserted
                        // hazard padding; extra wait states keep the read clear.
                        __builtin_amdgcn_sched_barrier(0);
                        asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if constexpr (KC == 2)
                        part[qt][0] += part[qt][1];
                } else if (ph == 1 || ph == 2) {
                    if constexpr (MODE == M_CLASSIFY) {
#pragma unroll
                        for (int e = 2 * (ph - 1); e < 2 * ph; ++e) {
                            // bytes: 0xFF where the projection is negative, else 0
                            const uint32_t t0 = __builtin_amdgcn_perm(sign_word(y[4 * e + 1]),
                                                                      sign_word(y[4 * e]), 0x0C0C0B09u);
                            const uint32_t t1 = __builtin_amdgcn_perm(sign_word(y[4 * e + 3]),
                                                                      sign_word(y[4 * e + 2]), 0x0B090C0Cu);
                            mb[qt][e] = (int)(t0 | t1);
                        }
                    } else {
                        uint32_t b = ph == 1 ? 0u : bits[qt];
#pragma unroll
                        for (int v = 8 * (ph - 1); v < 8 * ph; ++v)
                            b |= (sign_word(y[v]) >> 31) << (8 * (v >> 2) + (v & 3));
                        if (ph == 2) {
                            b <<= 4 * g;
                            b |= (uint32_t)__shfl_xor((int)b, 32);
                            const int nv = a.nd - w * kDimChunk;   // dimensions of this tile
                            if (nv < 32)
                                b &= nv > 0 ? (1u << nv) - 1u : 0u;
                        }
                        bits[qt] = b;
                    }
                } else if (ph == 3) {
                    if constexpr (MODE == M_CLASSIFY) {
#pragma unroll
                        for (int kt = 0; kt < KT; ++kt)
                            mma(dacc[kt][qt], cf[kt], mb[qt]);
                    } else {
                        const int64_t q = qbase + qt * 32 + (lane & 31);
                        if (g == 0 && q < a.n)
                            a.H32[q * a.ldh32 + w] = bits[qt];
                    }
                }
            }
        }
    };

    static __device__ __forceinline__ void run_epilogue(const Epilogue &epi)
    {
#pragma unroll
        for (int p = 0; p < kPhases; ++p)
            epi(p);
    }

    // The epilogue as a pass hook: phase p after K step p * SP.
    static constexpr int SP = KS >= 2 * kPhases ? 2 : 1;
    struct EpiHook {
        Epilogue epi;
        __device__ __forceinline__ void at(int s) const
        {
            if (s % SP == 0 && s / SP < kPhases)
                epi(s / SP);
        }
        __device__ __forceinline__ void tail() const
        {
#pragma unroll
            for (int p = (KS + SP - 1) / SP; p < kPhases; ++p)
                epi(p);
        }
    };
    template <class H1, class H2>
    struct Both {
        H1 h1;
        H2 h2;
        __device__ __forceinline__ void at(int s) const
        {
            h1.at(s);
            h2.at(s);
        }
        __device__ __forceinline__ void tail() const
        {
            h1.tail();
            h2.tail();
        }
    };

    // ------------------------------------------------------------ body
    // Runs the whole dimension loop for the queries of this workgroup.
    // Returns the class accumulators (classify mode) through dacc.
    static __device__ __forceinline__ void run(const EncodeArgs &a, uint8_t *smem, int64_t qblock,
                                               v16i (&dacc)[KT][QT])
    {
        if constexpr (DMA)
            run_dma(a, smem, qblock, dacc);
        else
            run_db(a, smem, qblock, dacc);
    }

    // Register-staged loop over a double-buffered LDS stage: step c
    // prefetches chunk c+1 into registers, multiplies chunk c while chunk
    // c-1's epilogue runs between its MFMAs, reads chunk c's class fragments
    // into registers, stores chunk c+1 into the other buffer and
    // synchronises once.  The two accumulator sets alternate, so the loop is
    // unrolled by two.
    static __device__ __forceinline__ void run_db(const EncodeArgs &a, uint8_t *smem, int64_t qblock,
                                                  v16i (&dacc)[KT][QT])
    {
        const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 5;
        const int64_t qbase = qblock + (int64_t)wave * QPW;
        const int ks_used = (a.F + KSTEP - 1) / KSTEP;
        const int npc = (ks_used * KSTEP + 15) / 16;
        const int NC = (a.nd + kDimChunk - 1) / kDimChunk;
        const bool colsum = CT == C_I8 && XF == 0 && a.x_type == X_UINT8;

        xfrag xr[QT][KS];
        load_x(xr, a, qbase, lane, ks_used);
        const acc_t x0[QT] = {};
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int qt = 0; qt < QT; ++qt)
                dacc[kt][qt] = v16i{};

        lds_u8 *L = (lds_u8 *)smem;
        lds_u8 *lp[2] = {L, L + kDimChunk * RSB};
        lds_u8 *lc[2] = {L + OFF_C, L + OFF_C + KT * 1024};
        lds_i32 *lcs[2] = {(lds_i32 *)(L + OFF_CS), (lds_i32 *)(L + OFF_CS) + kDimChunk};

        uint4 pr[MP];
        uint4 cr = make_uint4(0, 0, 0, 0);
        zero_tails(lp[0], lp[1], t, npc);
        stage_load(pr, a, 0, t, npc);
        if constexpr (MODE == M_CLASSIFY)
            cr = class_load(a, 0, t);
        stage_store(lp[0], lcs[0], pr, a, 0, t, npc, colsum);
        if constexpr (MODE == M_CLASSIFY)
            class_store(lc[0], cr, t);
        __syncthreads();

        v4i cf[KT];
        auto step = [&](int c, int b, Parts &cur, const auto &hook) {
            const bool more = c + 1 < NC;
            // prefetch the next chunk (the last step re-reads in-bounds data
            // and discards it, keeping the loop free of branches)
            stage_load(pr, a, c + 1, t, npc);
            if constexpr (MODE == M_CLASSIFY)
                cr = class_load(a, more ? c + 1 : c, t);
            tile_mma(cur, xr, lp[b], lcs[b], colsum, lane, hook, x0);
            if constexpr (MODE == M_CLASSIFY) {
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
                    cf[kt] = *(const lds_v4i *)(lc[b] + (kt * 64 + lane) * 16);
            }
            if (more) {
                stage_store(lp[b ^ 1], lcs[b ^ 1], pr, a, c + 1, t, npc, colsum);
                if constexpr (MODE == M_CLASSIFY)
                    class_store(lc[b ^ 1], cr, t);
            }
            __syncthreads();
        };

        Parts P0, P1;
        step(0, 0, P0, NoHook{});
        for (int c = 1;; c += 2) {
            if (c >= NC) {
                run_epilogue(Epilogue{a, P0, dacc, cf, c - 1, lane, g, qbase});
                break;
            }
            step(c, 1, P1, EpiHook{Epilogue{a, P0, dacc, cf, c - 1, lane, g, qbase}});
            if (c + 1 >= NC) {
                run_epilogue(Epilogue{a, P1, dacc, cf, c, lane, g, qbase});
                break;
            }
            step(c + 1, 0, P0, EpiHook{Epilogue{a, P1, dacc, cf, c, lane, g, qbase}});
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

    // ------------------------------------------------------------ DMA
    // Source of each of this lane's NIW loads: LDS unit u = (i * 4 + wave) *
    // 64 + lane of a stage is row u / UPR, piece u % UPR; the skew unit,
    // pieces past the features and rows past the chunk re-read piece 0 of an
    // in-bounds row (finite int8 against zero features, or slack).  Row r of
    // chunk c is dimension S_{c*CH + r}.  Byte offsets fit 32 bits: the
    // projection holds at most 65536 rows of at most 1024 + padding bytes.
    struct Loader {
        const EncodeArgs &a;
        uint32_t off0[NIW];   // offset of load i in chunk 0
        int rp[NIW];          // row | piece byte offset << 8
        uint32_t rstep, base, cbytes, lastrow;
        int NC, lane, wave;

        __device__ __forceinline__ Loader(const EncodeArgs &a_, int NC_, int npc, int wave_, int lane_)
            : a(a_), NC(NC_), lane(lane_), wave(wave_)
        {
            rstep = (uint32_t)a.stride * (uint32_t)a.ldp;
            base = (uint32_t)a.s0 * (uint32_t)a.ldp;
            cbytes = (uint32_t)CH * rstep;
            lastrow = base + (uint32_t)(a.nd - 1) * rstep;   // row of the last dimension
#pragma unroll
            for (int i = 0; i < NIW; ++i) {
                const int u = (i * kWaves + wave) * 64 + lane;
                int r = u / UPR, p = u % UPR;
                if (r >= CH) {
                    r = CH - 1;
                    p = 0;
                }
                const int pb = 16 * (p < npc ? p : 0);
                off0[i] = base + (uint32_t)r * rstep + (uint32_t)pb;
                rp[i] = r | (pb << 8);
            }
        }
        // Load i (< NIW + NCW) of chunk c, clamped to the last chunk: the
        // projection rows, then the class fragments (wave w loads class tiles
        // (w + 4j) % NCT; duplicate tiles write the same bytes).  In the
        // chunk holding the last dimension, rows past it re-read that row
        // (a select, not a branch: branches here would split the MFMA
        // sequence the loads are interleaved with into separate scheduling
        // regions).  The class table holds a whole number of chunks (zero
        // rows past nd).
        __device__ __forceinline__ void issue(int i, int c, lds_u8 *stage, lds_u8 *lcls) const
        {
            const int cc = c < NC ? c : NC - 1;
            if (i < NIW) {
                const int last = a.nd - 1 - cc * CH;      // >= CH - 1 except in the last chunk
                const uint32_t off = (rp[i] & 255) <= last ? off0[i] + (uint32_t)cc * cbytes
                                                            : lastrow + (uint32_t)(rp[i] >> 8);
                lds_dma16(a.P, off, stage + (i * kWaves + wave) * 1024);
            } else if constexpr (MODE == M_CLASSIFY) {
                const int tile = (wave + kWaves * (i - NIW)) % NCT;   // rt * KT + kt
                lds_dma16(a.ctab, (uint32_t)((cc * NCT + tile) * 1024 + lane * 16), lcls + tile * 1024);
            }
        }
    };
    static constexpr int NLOADS = NIW + (MODE == M_CLASSIFY ? NCW : 0);   // loads per wave per chunk

    // The loads of one chunk as a pass hook: load s after K step s.
    struct LoadHook {
        const Loader &ld;
        int c;
        lds_u8 *stage, *lcls;
        __device__ __forceinline__ void at(int s) const
        {
            if (s < NLOADS)
                ld.issue(s, c, stage, lcls);
        }
        __device__ __forceinline__ void tail() const
        {
#pragma unroll
            for (int s = KS; s < NLOADS; ++s)
                ld.issue(s, c, stage, lcls);
        }
    };

    // Wait until at most G of this wave's vector memory operations are in
    // flight (they complete in issue order, so everything older is done),
    // drain LDS operations, and meet the other waves.
    template <int G>
    static __device__ __forceinline__ void dma_barrier()
    {
        asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(G) : "memory");
    }

    // Staged loop: step c multiplies the RT row tiles of chunk c one after
    // the other, each with the previous row tile's epilogue between its
    // MFMAs (the first pass also issues the loads of the chunk NBUF - 1
    // ahead there), reads each tile's class fragments into registers right
    // after its pass, waits for chunk c+1's loads and synchronises once.
    // Three stages for one or two row tiles; two for three (96-dimension
    // chunks: 120 MFMAs per wave between barriers), whose next chunk's
    // loads then have one step to land.  Row tile passes rotate through RT
    // accumulator sets (two with RT = 1, the loop unrolled by two).
    static __device__ __forceinline__ void run_dma(const EncodeArgs &a, uint8_t *smem, int64_t qblock,
                                                   v16i (&dacc)[KT][QT])
    {
        static_assert(RT == 1 || RT == 2 || RT == 3, "one to three row tiles per chunk");
        const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 5;
        const int64_t qbase = qblock + (int64_t)wave * QPW;
        const int ks_used = (a.F + KSTEP - 1) / KSTEP;
        const int npc = (ks_used * KB + 15) / 16;   // 16-byte pieces of a row holding features
        const int NC = (a.nd + CH - 1) / CH;
        // loads issued per step after those of the chunk waited for (stores
        // of the encode epilogue are not counted: waiting for more is safe);
        // with two stages the chunk waited for is the one issued last
        constexpr int G = NBUF == 3 ? NLOADS : 0;

        xfrag xr[QT][KS];
        load_x(xr, a, qbase, lane, ks_used);
        acc_t x0[QT];
        shift_start(x0, xr, a.poff);
        if constexpr (kShift && CT == C_FP8) {
            // the E4M3 start values come from 16-pass MFMAs: wait states
            // before anything reads them (as in the epilogue)
            __builtin_amdgcn_sched_barrier(0);
            asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int qt = 0; qt < QT; ++qt)
                dacc[kt][qt] = v16i{};

        lds_u8 *L = (lds_u8 *)smem;
        auto lp = [&](int i) { return L + i * SSZ; };
        auto lc = [&](int i) { return L + OFF_C + i * (NCT * 1024); };
        const Loader ld(a, NC, npc, wave, lane);
#pragma unroll
        for (int c = 0; c < NBUF - 1; ++c)
#pragma unroll
            for (int i = 0; i < NLOADS; ++i)
                ld.issue(i, c, lp(c), lc(c));
        dma_barrier<G>();

        v4i cf[KT];
        int b = 0;   // stage of the chunk being multiplied
        auto read_cf = [&](int rt) {
            if constexpr (MODE == M_CLASSIFY) {
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
                    cf[kt] = *(const lds_v4i *)(lc(b) + ((rt * KT + kt) * 64 + lane) * 16);
            }
        };
        // one row-tile pass of the current chunk into cur
        auto pass = [&](int rt, Parts &cur, const auto &hook) {
            tile_mma(cur, xr, lp(b) + rt * kDimChunk * RSB, nullptr, false, lane, hook, x0);
            read_cf(rt);
        };
        auto loads = [&](int c) {   // loads of chunk c + NBUF - 1 into the free stage
            if constexpr (NBUF == 3) {
                const int b2 = b == 0 ? 2 : b - 1;   // (b + 2) % 3
                return LoadHook{ld, c + 2, lp(b2), lc(b2)};
            } else {
                return LoadHook{ld, c + 1, lp(b ^ 1), lc(b ^ 1)};
            }
        };
        auto epi = [&](Parts &prev, int w) { return EpiHook{Epilogue{a, prev, dacc, cf, w, lane, g, qbase}}; };
        typedef Both<EpiHook, LoadHook> EpiLoad;
        typedef Both<NoHook, LoadHook> JustLoad;
        auto finish_step = [&]() {
            dma_barrier<G>();
            b = b == NBUF - 1 ? 0 : b + 1;
        };

        Parts P0, P1;
        if constexpr (RT == 3) {
            Parts P2;
            pass(0, P0, JustLoad{NoHook{}, loads(0)});
            pass(1, P1, epi(P0, 0));
            pass(2, P2, epi(P1, 1));
            finish_step();
            for (int c = 1; c < NC; ++c) {
                pass(0, P0, EpiLoad{epi(P2, 3 * c - 1), loads(c)});
                pass(1, P1, epi(P0, 3 * c));
                pass(2, P2, epi(P1, 3 * c + 1));
                finish_step();
            }
            run_epilogue(Epilogue{a, P2, dacc, cf, 3 * NC - 1, lane, g, qbase});
        } else if constexpr (RT == 2) {
            pass(0, P0, JustLoad{NoHook{}, loads(0)});
            pass(1, P1, epi(P0, 0));
            finish_step();
            for (int c = 1; c < NC; ++c) {
                pass(0, P0, EpiLoad{epi(P1, 2 * c - 1), loads(c)});
                pass(1, P1, epi(P0, 2 * c));
                finish_step();
            }
            run_epilogue(Epilogue{a, P1, dacc, cf, 2 * NC - 1, lane, g, qbase});
        } else {
            pass(0, P0, JustLoad{NoHook{}, loads(0)});
            finish_step();
            for (int c = 1;; c += 2) {
                if (c >= NC) {
                    run_epilogue(Epilogue{a, P0, dacc, cf, c - 1, lane, g, qbase});
                    break;
                }
                pass(0, P1, EpiLoad{epi(P0, c - 1), loads(c)});
                finish_step();
                if (c + 1 >= NC) {
                    run_epilogue(Epilogue{a, P1, dacc, cf, c, lane, g, qbase});
                    break;
                }
                pass(0, P0, EpiLoad{epi(P1, c), loads(c + 1)});
                finish_step();
            }
        }
        // no load may still be writing this workgroup's LDS when it exits
        __builtin_amdgcn_s_waitcnt(0);
        if constexpr (MODE == M_ENCODE && RT == 1) {
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
