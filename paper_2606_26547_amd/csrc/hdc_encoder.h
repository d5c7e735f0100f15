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

template <int CT, int XF, int QT, int KS, int KT, int MODE, bool PIPE = false>
struct Encoder {
    typedef Tr<CT> T;
    typedef typename T::frag frag;
    typedef typename T::acc acc_t;
    static constexpr int KSTEP = T::KSTEP;
    static constexpr int KB = KSTEP * T::ESZ;              // LDS bytes per K-step per row
    static constexpr int RSB = KS * KB + 16;               // LDS row stride (16 B skew)
    static constexpr int PIECES = (KS * KSTEP + 15) / 16;  // 16-byte int8 pieces per row (max)
    static constexpr int MP = (PIECES + 7) / 8;            // pieces per thread (8 threads / row)
    // Three LDS stages (software-pipelined loop) when they fit beside a second
    // workgroup's worth of headroom, else two (plain double buffering).
    static constexpr int NBUF = PIPE ? 3 : 2;
    static constexpr int OFF_C = NBUF * kDimChunk * RSB;
    static constexpr int OFF_CS = OFF_C + (MODE == M_CLASSIFY ? NBUF * KT * 1024 : 0);
    static constexpr int LDS = OFF_CS + NBUF * kDimChunk * 4;
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
                frag f = load_frag(a, qc, v ? s : 0, g);
                if (!v)
                    f = frag{};
                xr[qt][s] = f;
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
            } else if constexpr (CT == C_FP8) {
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
    // Fixed-length, branch-free K loop over the chunk in LDS with the next
    // projection fragment read while the current one is multiplied (steps
    // past the feature count read zero-filled LDS against zero features).
    struct NoHook {
        __device__ __forceinline__ void operator()(int) const {}
    };
    static constexpr int kMaxPhases = 8;   // epilogue phases a hook may run

    static __device__ __forceinline__ void chunk_mma(acc_t (&acc)[QT], const frag (&xr)[QT][KS],
                                                     const lds_u8 *lp, int lane)
    {
        chunk_mma(acc, xr, lp, lane, NoHook{});
    }

    // hook(p) runs phase p of another chunk's epilogue right after the
    // MFMAs of step p, so its VALU work issues while the matrix core is busy;
    // phases past the last step run after the loop.
    template <class Hook>
    static __device__ __forceinline__ void chunk_mma(acc_t (&acc)[QT], const frag (&xr)[QT][KS],
                                                     const lds_u8 *lp, int lane, const Hook &hook)
    {
        const int g = lane >> 5, row = lane & 31;
        // A dependent MFMA chain issues at half rate on gfx950 (the result
        // latency is twice the issue interval), so with one query tile the
        // K steps alternate between two accumulators (KC chains) that are
        // added at the end: exact for int32, and order-free for the float
        // rungs on integer-valued features (sums below 2^24).
        constexpr int KC = (QT == 1 && KS >= 2) ? 2 : 1;
        acc_t part[QT][KC];
#pragma unroll
        for (int qt = 0; qt < QT; ++qt)
#pragma unroll
            for (int k = 0; k < KC; ++k)
                part[qt][k] = acc_t{};
        const lds_u8 *base = lp + row * RSB + g * (KB / 2);
        // PD fragments in flight; the scheduling barriers keep each read
        // PD steps ahead of its use instead of next to it.
        constexpr int PDW = (CT == C_I8 && QT == 1) ? 4 : (CT == C_F32 ? 4 : 2);
        constexpr int PD = KS < PDW ? KS : PDW;
        frag f[PD];
#pragma unroll
        for (int s = 0; s < PD; ++s)
            f[s] = *(const HDC_LDS frag *)(base + s * KB);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const frag cur = f[s % PD];
            if (s + PD < KS)
                f[s % PD] = *(const HDC_LDS frag *)(base + (s + PD) * KB);
#pragma unroll
            for (int qt = 0; qt < QT; ++qt)
                mma(part[qt][s % KC], cur, xr[qt][s]);
            hook(s);
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (CT == C_FP8) {
            // The 16-pass E4M3 MFMA's last accumulator register was observed
            // to be read one wait state too early by the compiler-inserted
            // hazard padding (a wrong sign in register 15 right after the
            // loop); sleeping ~64 clocks keeps every read past the window.
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_sleep(1);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            acc[qt] = part[qt][0];
            if constexpr (KC == 2)
                acc[qt] += part[qt][1];
        }
#pragma unroll
        for (int p = KS; p < kMaxPhases; ++p)
            hook(p);
    }

    // Sign words of one tile, with the uint8 column-sum correction.
    static __device__ __forceinline__ void signs(uint32_t (&w)[16], const acc_t &acc, const lds_i32 *lcs,
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
        if constexpr (NBUF == 3)
            run_pipe(a, smem, qblock, dacc);
        else
            run_db(a, smem, qblock, dacc);
    }

    // Epilogue of one chunk split into phases (see chunk_mma's hook).
    //   classify: phase 0 reads the class fragments; per query tile qt,
    //             phases 1+3qt and 2+3qt turn the signs into {0,-1} bytes
    //             and phase 3+3qt runs the Hamming MFMAs.
    //   encode:   per query tile, phase 3qt packs the first 8 signs, 1+3qt
    //             the rest (and joins the lane halves), 2+3qt stores.
    struct Epilogue {
        const EncodeArgs &a;
        const acc_t (&acc)[QT];
        v16i (&dacc)[KT][QT];
        const lds_u8 *lc;
        const lds_i32 *lcs;
        int c, lane, g;
        int64_t qbase;
        bool colsum;
        mutable v4i cf[KT];
        mutable v4i mb[QT];
        mutable uint32_t bits[QT];

        __device__ __forceinline__ uint32_t sw(int qt, int v) const
        {
            if constexpr (CT == C_I8) {
                int y = acc[qt][v];
                if (colsum)
                    y += 128 * lcs[8 * (v >> 2) + 4 * g + (v & 3)];
                return sign_word(y);
            } else {
                return sign_word(acc[qt][v]);
            }
        }

        __device__ __forceinline__ void operator()(int p) const
        {
            if constexpr (MODE == M_CLASSIFY) {
                if (p == 0) {
#pragma unroll
                    for (int kt = 0; kt < KT; ++kt)
                        cf[kt] = *(const lds_v4i *)(lc + (kt * 64 + lane) * 16);
                    return;
                }
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) {
                    const int ph = p - 1 - 3 * qt;
                    if (ph == 0 || ph == 1) {
#pragma unroll
                        for (int e = 2 * ph; e < 2 * ph + 2; ++e) {
                            // bytes: 0xFF where the projection is negative, else 0
                            uint32_t t0 = __builtin_amdgcn_perm(sw(qt, 4 * e + 1), sw(qt, 4 * e), 0x0C0C0B09u);
                            uint32_t t1 = __builtin_amdgcn_perm(sw(qt, 4 * e + 3), sw(qt, 4 * e + 2), 0x0B090C0Cu);
                            mb[qt][e] = (int)(t0 | t1);
                        }
                    } else if (ph == 2) {
#pragma unroll
                        for (int kt = 0; kt < KT; ++kt)
                            mma(dacc[kt][qt], cf[kt], mb[qt]);
                    }
                }
            } else {
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) {
                    const int ph = p - 3 * qt;
                    if (ph == 0 || ph == 1) {
                        uint32_t b = ph == 0 ? 0u : bits[qt];
#pragma unroll
                        for (int v = 8 * ph; v < 8 * ph + 8; ++v)
                            b |= (sw(qt, v) >> 31) << (8 * (v >> 2) + (v & 3));
                        if (ph == 1) {
                            b <<= 4 * g;
                            b |= (uint32_t)__shfl_xor((int)b, 32);
                        }
                        bits[qt] = b;
                    } else if (ph == 2) {
                        const int64_t q = qbase + qt * 32 + (lane & 31);
                        if (g == 0 && q < a.n)
                            a.H32[q * a.ldh32 + c] = bits[qt];
                    }
                }
            }
        }
    };

    // Software-pipelined loop over a ring of three LDS stages: iteration c
    // prefetches chunk c+2 into registers, multiplies chunk c+1 while chunk
    // c's epilogue runs between its MFMAs, stores chunk c+2 into the stage
    // that chunk c-1 used, and synchronises once.  The two accumulator sets
    // alternate, so the loop is unrolled by two.
    static __device__ __forceinline__ void run_pipe(const EncodeArgs &a, uint8_t *smem, int64_t qblock,
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

        lds_u8 *L = (lds_u8 *)smem;
        auto lp = [&](int i) { return L + i * (kDimChunk * RSB); };
        auto lc = [&](int i) { return L + OFF_C + i * (KT * 1024); };
        auto lcs = [&](int i) { return (lds_i32 *)(L + OFF_CS) + i * kDimChunk; };

        uint4 pr[MP];
        uint4 cr = make_uint4(0, 0, 0, 0);
        zero_tails(lp(0), lp(1), t, npc);
        zero_tails(lp(2), lp(2), t, npc);
        stage_load(pr, a, 0, t, npc);
        if constexpr (MODE == M_CLASSIFY)
            cr = class_load(a, 0, t);
        stage_store(lp(0), lcs(0), pr, a, 0, t, npc, colsum);
        if constexpr (MODE == M_CLASSIFY)
            class_store(lc(0), cr, t);
        stage_load(pr, a, 1, t, npc);
        if constexpr (MODE == M_CLASSIFY)
            cr = class_load(a, NC > 1 ? 1 : 0, t);
        if (NC > 1) {
            stage_store(lp(1), lcs(1), pr, a, 1, t, npc, colsum);
            if constexpr (MODE == M_CLASSIFY)
                class_store(lc(1), cr, t);
        }
        __syncthreads();

        acc_t A[QT], B[QT];
        chunk_mma(A, xr, lp(0), lane);

        // one pipelined iteration: epilogue of chunk c (accumulators cur,
        // stage bc) interleaved with the MFMAs of chunk c+1 into nxt
        auto body = [&](int c, int bc, const acc_t (&cur)[QT], acc_t (&nxt)[QT]) {
            const int b1 = bc == 2 ? 0 : bc + 1, b2 = b1 == 2 ? 0 : b1 + 1;
            stage_load(pr, a, c + 2, t, npc);
            if constexpr (MODE == M_CLASSIFY)
                cr = class_load(a, c + 2 < NC ? c + 2 : NC - 1, t);
            Epilogue epi{a, cur, dacc, lc(bc), lcs(bc), c, lane, g, qbase, colsum};
            chunk_mma(nxt, xr, lp(b1), lane, epi);
            if (c + 2 < NC) {
                stage_store(lp(b2), lcs(b2), pr, a, c + 2, t, npc, colsum);
                if constexpr (MODE == M_CLASSIFY)
                    class_store(lc(b2), cr, t);
            }
            __syncthreads();
        };
        auto last = [&](int c, int bc, const acc_t (&cur)[QT]) {
            Epilogue epi{a, cur, dacc, lc(bc), lcs(bc), c, lane, g, qbase, colsum};
#pragma unroll
            for (int p = 0; p < kMaxPhases; ++p)
                epi(p);
        };

        int bc = 0;
        for (int c = 0;; c += 2) {
            if (c + 1 >= NC) {
                last(c, bc, A);
                break;
            }
            body(c, bc, A, B);
            bc = bc == 2 ? 0 : bc + 1;
            if (c + 2 >= NC) {
                last(c + 1, bc, B);
                break;
            }
            body(c + 1, bc, B, A);
            bc = bc == 2 ? 0 : bc + 1;
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

    // Plain double-buffered loop (used when three stages do not fit).
    static __device__ __forceinline__ void run_db(const EncodeArgs &a, uint8_t *smem, int64_t qblock,
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

        for (int c = 0; c < NC; ++c) {
            const int b = c & 1;
            const bool more = c + 1 < NC;
            // prefetch the next chunk (the last iteration re-reads in-bounds
            // data and discards it, keeping the loop free of branches)
            stage_load(pr, a, c + 1, t, npc);
            if constexpr (MODE == M_CLASSIFY)
                cr = class_load(a, more ? c + 1 : c, t);
            acc_t acc[QT];
            chunk_mma(acc, xr, lp[b], lane);
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
                    cf[kt] = *(const lds_v4i *)(lc[b] + (kt * 64 + lane) * 16);
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
