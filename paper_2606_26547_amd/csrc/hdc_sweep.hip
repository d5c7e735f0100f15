// hdc_eval_configs: one persistent launch that classifies the same queries
// under many approximation configurations (the inner loop of the tuning
// system: run each candidate, read back its accuracy and time).
//
// The host validates the configurations, orders them longest first, lays
// out their work items and finds the distinct dimension sets (configurations
// of the same start, end and stride share one class operand), and sends all
// of it up in one copy.  Workspace layout (all offsets 256-byte aligned):
//   [0]            queue counter (uint32)
//   [256]          slot descriptors, ncfg x SlotDesc
//   [..]           slot order (longest first), ncfg x int32
//   [..]           first work item of each slot in that order, ncfg + 1 x int32
//   [..]           per-slot counters (correct, n, device ticks), zeroed
//   [..]           distinct dimension sets, up to ncfg x TableDesc
//   [..]           per-slot results as returned (correct, n, device_us)
//   [..]           class operand regions of fixed size, one per distinct
//                  dimension set (chunks(D) * KT KiB table + 128 int32
//                  popcounts)
//   [..]           shared search items, up to ncfg x ShItem
//   [..]           shared end counters (correct, device ticks), zeroed
//   [..]           projection rows converted to E4M3 (direct-staged body)
//   [..]           packed encodings of the shared path: one region per
//                  encoding (int8, E4M3), kShQueries rows of ceil(D / 64)
//                  words
// Work item i belongs to the slot whose item range holds it (a binary search
// over the item offsets); a workgroup takes items from the queue until it is
// exhausted, so every workgroup reaches the exit whatever the grid size.
//
// Shared configurations (tile SV_SHARED) skip the persistent kernel.  The
// encoding of one dimension depends on that dimension's projection row and
// the queries only, and so does its class bit; the configurations of one
// compute type therefore take their distances from one encoding of the
// union of their dimension sets (64-aligned from below), by masked Hamming
// distance (bf16 configurations from the int8 encoding, which equals theirs
// for integer features).  Configurations with the same start and stride form a chain
// whose sets are prefixes of each other: one pass over the chain's words
// gives every end's distances on the way.
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "hdc_encoder.h"

namespace hdc {

struct SlotDesc {
    int32_t s0, stride, nd, ct;   // ct < 0: invalid configuration (no work)
    int32_t iq;                   // work items: 1 = 128 queries, 2 = 256, 3 = 256 on the direct-staged body
    int32_t tiles;                // work items of the slot
    int32_t table;                // its class operand (distinct dimension set)
    int32_t pad;
};

// A distinct dimension set.
struct TableDesc {
    int32_t s0, stride, nd, pad;
};

// Per-slot counters of the persistent kernel.
struct SlotCount {
    int32_t correct, n;
    uint64_t ticks;
};

// Shared path: ends per search item, words per LDS chunk, queries per pass.
constexpr int kShEnds = 16;
constexpr int kShWords = 16;
constexpr int kShQueries = 4096;

// A search item: one chain (compute type region, start, stride) and up to
// kShEnds of its set ends, ascending; it reads absolute words [a0, a1).
struct ShItem {
    int32_t reg;                  // encoding region
    int32_t s0, stride;
    int32_t wlo;                  // absolute word of the region's column 0
    int32_t a0, a1;
    int32_t nend, pad;
    int32_t end[kShEnds];         // one past the last dimension of each set
    int32_t slot[kShEnds];        // its end counter
};

struct EndCount {
    int32_t correct, pad;
    uint64_t ticks;
};

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Class tiles compiled into the sweep kernel: 1 (K <= 32) or 4 (K <= 128).
// A slot's table holds whole pairs of 32-dimension chunks (the direct-staged
// 2x2 body reads them in pairs; the pad chunk is zero).
inline size_t sweep_table_bytes(int D, int K) { return (size_t)table_chunks(D) * sweep_kt(K) * 1024; }

// Rows of the projection converted for the direct-staged E4M3 body: +-1 as
// E4M3 bytes, pitch ldp_conv (F rounded up to 64), pad columns 0.
inline size_t conv_pitch(int F) { return (size_t)(F + 63) / 64 * 64; }

struct SweepLayout {
    size_t off_desc, off_order, off_items, off_count, off_tabs, off_sh, off_end, off_res, off_regions, region;
    size_t off_p8, ldp_conv, off_h, hreg, wd, total;
    SweepLayout(int ncfg, int F, int D, int K)
    {
        off_desc = 256;
        off_order = align256(off_desc + (size_t)ncfg * sizeof(SlotDesc));
        off_items = align256(off_order + (size_t)ncfg * 4);
        off_count = align256(off_items + (size_t)(ncfg + 1) * 4);
        off_tabs = align256(off_count + (size_t)ncfg * sizeof(SlotCount));
        off_sh = align256(off_tabs + (size_t)ncfg * sizeof(TableDesc));
        off_end = align256(off_sh + (size_t)ncfg * sizeof(ShItem));
        off_res = align256(off_end + (size_t)ncfg * sizeof(EndCount));
        off_regions = align256(off_res + (size_t)ncfg * sizeof(hdc_config_result));
        region = align256(sweep_table_bytes(D, K) + 128 * 4);
        ldp_conv = conv_pitch(F);
        off_p8 = align256(off_regions + region * (size_t)ncfg);
        wd = (size_t)(D + 63) / 64;
        hreg = align256((size_t)kShQueries * wd * 8);
        off_h = align256(off_p8 + (size_t)D * ldp_conv);
        total = off_h + 2 * hreg;
    }
};

size_t sweep_workspace_bytes(int32_t ncfg, int32_t F, int32_t D, int32_t K)
{
    if (ncfg <= 0 || F <= 0 || D <= 0 || K <= 0 || K > kMaxK)
        return 0;
    return SweepLayout(ncfg, F, D, K).total;
}

// The converted projection rows (E4M3 +-1.0, zero past F).
__global__ __launch_bounds__(256) void k_sweep_convert(const int8_t *__restrict__ P, int64_t ldp, int D, int F,
                                                       uint8_t *__restrict__ ws, SweepLayout L)
{
    uint8_t *p8 = ws + L.off_p8;
    const int64_t total = (int64_t)D * (int64_t)L.ldp_conv;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t d = i / (int64_t)L.ldp_conv, f = i % (int64_t)L.ldp_conv;
        p8[i] = f < F ? (P[d * ldp + f] < 0 ? 0xB8u : 0x38u) : 0u;
    }
}

// Per-slot results in the returned form: device time in microseconds.
__global__ __launch_bounds__(256) void k_sweep_results(int ncfg, const uint8_t *__restrict__ ws, SweepLayout L,
                                                       double us_per_tick)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ncfg)
        return;
    const SlotCount c = ((const SlotCount *)(ws + L.off_count))[i];
    const SlotDesc d = ((const SlotDesc *)(ws + L.off_desc))[i];
    hdc_config_result r;
    r.n = c.n;
    if (d.iq == SV_SHARED && d.ct >= 0) {
        const EndCount e = ((const EndCount *)(ws + L.off_end))[d.table];
        r.correct = e.correct;
        r.device_us = (double)e.ticks * us_per_tick;
    } else {
        r.correct = c.correct;
        r.device_us = (double)c.ticks * us_per_tick;
    }
    ((hdc_config_result *)(ws + L.off_res))[i] = r;
}

// Class operand tables of every slot (same layout as hdc_classify's).
__global__ __launch_bounds__(256) void k_sweep_tables(const uint64_t *__restrict__ C, int K, int64_t ldc,
                                                      uint8_t *__restrict__ ws, SweepLayout L, int KT,
                                                      int64_t per_slot)
{
    const int t = blockIdx.y;
    const TableDesc s = ((const TableDesc *)(ws + L.off_tabs))[t];
    int8_t *tab = (int8_t *)(ws + L.off_regions + L.region * t);
    // whole pairs of chunks; chunks past nd are written as zeros
    const int64_t total = (int64_t)((s.nd + 2 * kDimChunk - 1) / (2 * kDimChunk)) * 2 * KT * 64;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total && idx < per_slot;
         idx += (int64_t)gridDim.x * 256) {
        const int lane = (int)(idx & 63);
        const int kt = (int)((idx >> 6) % KT);
        const int64_t c = (idx >> 6) / KT;
        const int k = kt * 32 + (lane & 31), g = lane >> 5;
        uint32_t o[4] = {0, 0, 0, 0};
        if (k < K) {
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                const int64_t dl = c * kDimChunk + 8 * (b >> 2) + 4 * g + (b & 3);
                if (dl < s.nd) {
                    const int64_t d = s.s0 + dl * s.stride;
                    const uint32_t bit = (uint32_t)(C[k * ldc + (d >> 6)] >> (d & 63)) & 1u;
                    o[b >> 2] |= (bit ? 0xffu : 0x01u) << (8 * (b & 3));
                }
            }
        }
        *(uint4 *)(tab + idx * 16) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

__global__ __launch_bounds__(256) void k_sweep_popc(const uint64_t *__restrict__ C, int K, int64_t ldc,
                                                    uint8_t *__restrict__ ws, SweepLayout L, size_t table_bytes)
{
    __shared__ int part[256];
    const int t = blockIdx.y, k = blockIdx.x;
    const TableDesc s = ((const TableDesc *)(ws + L.off_tabs))[t];
    int32_t *popc = (int32_t *)(ws + L.off_regions + L.region * t + table_bytes);
    int acc = 0;
    if (k < K)
        for (int64_t dl = threadIdx.x; dl < s.nd; dl += 256) {
            const int64_t d = s.s0 + dl * s.stride;
            acc += (int)((C[k * ldc + (d >> 6)] >> (d & 63)) & 1u);
        }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        popc[k] = part[0];
}

// Bits of absolute word a that belong to the set {s0 + i * stride} below
// `end`: the first one at or after s0 on the stride's grid, then doubled
// along the stride.
__device__ __forceinline__ uint64_t chain_mask(int a, int s0, int stride, int end)
{
    const int base = 64 * a;
    if (base + 64 <= s0 || base >= end)
        return 0;
    int j0 = s0 - base;
    if (j0 < 0) {
        const int r = (base - s0) % stride;
        j0 = r ? stride - r : 0;
    }
    if (j0 >= 64)
        return 0;
    uint64_t m = 1ull << j0;
    for (int sh = stride; sh < 64; sh <<= 1)
        m |= m << sh;
    const int rem = end - base;
    return rem < 64 ? m & ((1ull << rem) - 1) : m;
}

// Shared search: workgroup (query block of 64, item).  Each of the NW
// waves takes KCW classes of the same 64 queries (one query per lane).
// Chunks of kShWords words of the queries' encodings and of the class words
// go through registers (the next chunk's loads are in flight while the
// current one is counted) into LDS, both cut to the chain's set by masks
// computed one chunk ahead.  Per word, a lane adds popcount(h ^ c) to each
// of its classes' distances.  At the last word of a set's end, the
// distances up to that end (that word cut below the end) are ranked by the
// key distance * 128 + class, whose minimum is the first smallest distance;
// the waves meet in an LDS minimum.  The 64 labels of each end are then
// compared with the truth and counted into the end's counter.
template <int KCW, int NW>
__global__ __launch_bounds__(64 * NW) void k_sweep_shared(const uint64_t *__restrict__ C, int K, int64_t ldc,
                                                          const int32_t *__restrict__ truth, int nq,
                                                          uint8_t *__restrict__ ws, SweepLayout L)
{
    constexpr int T = 64 * NW;
    constexpr int CW = kShWords * NW * KCW / T;      // class words per thread and chunk
    constexpr int HW = kShWords * 64 / T;            // encoding words per thread and chunk
    static_assert(CW >= 1 && HW >= 1 && kShWords % HW == 0, "chunk split");
    __shared__ uint64_t cm[kShWords][NW * KCW];
    __shared__ uint64_t hs[64][kShWords + 1];
    __shared__ uint64_t msk[2][kShWords];
    __shared__ int best[kShEnds][64];
    __shared__ int ends[kShEnds];
    const ShItem &it = ((const ShItem *)(ws + L.off_sh))[blockIdx.y];
    const uint64_t *H = (const uint64_t *)(ws + L.off_h + L.hreg * it.reg);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int qb = blockIdx.x * 64;
    const int nend = it.nend, s0 = it.s0, stride = it.stride, wlo = it.wlo, a0 = it.a0, a1 = it.a1;
    const int end_max = it.end[nend - 1];
    const uint64_t t0 = wall_clock64();
    for (int i = tid; i < kShEnds * 64; i += T)
        best[i >> 6][i & 63] = 0x7fffffff;
    if (tid < nend)
        ends[tid] = it.end[tid];
    // this thread's share of a chunk: words hw .. hw + HW - 1 of query row
    // hq, and class words (word i % kShWords, class i / kShWords) for
    // i = tid + T r
    const int hq = tid / (kShWords / HW), hw = HW * (tid % (kShWords / HW));
    const bool hrow = qb + hq < nq;
    const uint64_t *hp = H + (int64_t)(qb + hq) * L.wd - wlo + hw;
    uint64_t rh[HW], rc[CW];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int x = 0; x < HW; ++x)
            rh[x] = hrow && c0 + hw + x < a1 ? hp[c0 + x] : 0;
#pragma unroll
        for (int r = 0; r < CW; ++r) {
            const int i = tid + T * r, ww = i & (kShWords - 1), k = i / kShWords;
            rc[r] = k < K && c0 + ww < a1 ? C[(int64_t)k * ldc + c0 + ww] : 0;
        }
    };
    if (tid < kShWords)
        msk[0][tid] = chain_mask(a0 + tid, s0, stride, end_max);
    fetch(a0);
    __syncthreads();
    const int kb = wave * KCW;
    int acc[KCW];
#pragma unroll
    for (int j = 0; j < KCW; ++j)
        acc[j] = 0;
    int e = 0;    // next end to emit, and the word of its last dimension
    int elw = __builtin_amdgcn_readfirstlane((ends[0] - 1) / 64);
    int b = 0;
    for (int c0 = a0; c0 < a1; c0 += kShWords, b ^= 1) {
        const int nw = a1 - c0 < kShWords ? a1 - c0 : kShWords;
#pragma unroll
        for (int x = 0; x < HW; ++x)
            hs[hq][hw + x] = rh[x] & msk[b][hw + x];
#pragma unroll
        for (int r = 0; r < CW; ++r) {
            const int i = tid + T * r, ww = i & (kShWords - 1), k = i / kShWords;
            cm[ww][k] = rc[r] & msk[b][ww];
        }
        if (c0 + kShWords < a1) {
            if (tid < kShWords)
                msk[b ^ 1][tid] = chain_mask(c0 + kShWords + tid, s0, stride, end_max);
            fetch(c0 + kShWords);
        }
        __syncthreads();
        for (int w = 0; w < nw;) {
            if (c0 + w == elw) {
                // sets whose last dimension lies in this word
                const int a = c0 + w;
                const uint64_t h = hs[lane][w];
                while (e < nend && (ends[e] - 1) / 64 == a) {
                    const int rem = ends[e] - 64 * a;
                    const uint64_t pm = rem >= 64 ? ~0ull : (1ull << rem) - 1;
                    int key = 0x7fffffff;
#pragma unroll
                    for (int j = 0; j < KCW; ++j) {
                        const int k = kb + j;
                        const int d = acc[j] + (int)__popcll((h ^ cm[w][k]) & pm);
                        if (k < K)
                            key = min(key, d * 128 + k);
                    }
                    atomicMin(&best[e][lane], key);
                    ++e;
                }
                elw = e < nend ? __builtin_amdgcn_readfirstlane((ends[e] - 1) / 64) : 0x7fffffff;
#pragma unroll
                for (int j = 0; j < KCW; ++j)
                    acc[j] += (int)__popcll(h ^ cm[w][kb + j]);
                ++w;
                continue;
            }
            // words up to the next set's last word: four at a time, their
            // LDS reads issued together
            const int stop = elw - c0 < nw ? elw - c0 : nw;
            for (; w + 4 <= stop; w += 4) {
                uint64_t h[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    h[u] = hs[lane][w + u];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int j = 0; j < KCW; ++j)
                        acc[j] += (int)__popcll(h[u] ^ cm[w + u][kb + j]);
            }
            for (; w < stop; ++w) {
                const uint64_t h = hs[lane][w];
#pragma unroll
                for (int j = 0; j < KCW; ++j)
                    acc[j] += (int)__popcll(h ^ cm[w][kb + j]);
            }
        }
        __syncthreads();    // the chunk's LDS reads are done
    }
    EndCount *cnt = (EndCount *)(ws + L.off_end);
    const uint64_t dt = wall_clock64() - t0;
    for (int x = wave; x < nend; x += NW) {
        const int q = qb + lane;
        const bool ok = q < nq && (best[x][lane] & 127) == truth[q];
        const uint64_t m = __ballot(ok);
        if (lane == 0) {
            if (m)
                atomicAdd(&cnt[it.slot[x]].correct, (int)__popcll(m));
            atomicAdd((unsigned long long *)&cnt[it.slot[x]].ticks, (unsigned long long)dt);
        }
    }
}

// One encoder pass of QT query tiles per wave over the queries from qblock,
// adding the correct labels to the slot's count.
template <int CT, int QT, int KS, int KT>
__device__ __forceinline__ void sweep_pass(EncodeArgs &a, uint8_t *smem, int64_t qblock, const int32_t *truth,
                                           SlotCount *res)
{
    typedef Encoder<CT, 0, QT, KS, KT, M_CLASSIFY, 1> E;
    v16i dacc[KT][QT];
    E::run(a, smem, qblock, dacc);
    int32_t lab[QT];
    E::finish(a, qblock, dacc, lab);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int qt = 0; qt < QT; ++qt) {
        const int64_t q = qblock + (int64_t)wave * E::QPW + qt * 32 + (lane & 31);
        const bool ok = lane < 32 && q < a.n && lab[qt] == truth[q];
        const uint64_t m = __ballot(ok);
        if (lane == 0 && m)
            atomicAdd(&res->correct, (int)__popcll(m));
    }
}

// Two int8 query tiles per wave fit the sweep's one wave per SIMD up to 20
// K steps (640 features).
constexpr bool sweep_qt2(int ct, int ks, int kt) { return ct == C_I8 && ks <= 20 && kt == 1; }

// Direct-staged bodies of the sweep (work items of 256 queries): up to 640
// features and one class tile, the int8 path (int8 features) and the E4M3
// path on the fused classifier's 2x2 shape; the E4M3 body reads projection
// rows converted once per launch.  (A bf16 body would hold one query tile
// only, beside its 40-step operand: one LDS fragment per MFMA then keeps
// LDS, not the matrix cores, busy, and it measured slower than register
// staging; bf16 configurations stage through registers.)
constexpr bool dma_sweep_fits(int ct, int ks, int kt)
{
    return kt == 1 && (ct == C_I8 || ct == C_FP8) && ks * kstep_of(ct) <= 640;
}

template <int CT, int KS, int KT, int QT, int RT>
__device__ __forceinline__ void sweep_pass_dma(EncodeArgs &a, uint8_t *smem, int64_t qblock, const int32_t *truth,
                                               SlotCount *res)
{
    typedef Encoder<CT, 0, QT, KS, KT, M_CLASSIFY, 1, true, RT> E;
    v16i dacc[KT][QT];
    E::run(a, smem, qblock, dacc);
    int32_t lab[QT];
    E::finish(a, qblock, dacc, lab);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int qt = 0; qt < QT; ++qt) {
        const int64_t q = qblock + (int64_t)wave * E::QPW + qt * 32 + (lane & 31);
        const bool ok = lane < 32 && q < a.n && lab[qt] == truth[q];
        const uint64_t m = __ballot(ok);
        if (lane == 0 && m)
            atomicAdd(&res->correct, (int)__popcll(m));
    }
}

// A work item of 128 queries (IQ = 1) or 256 (IQ = 2, 3).  With IQ = 2,
// int8 slots take both query tiles per wave in one pass where the registers
// allow (each projection fragment staged once for 256 queries), other slots
// run two passes; IQ = 3 runs on the direct-staged bodies where they are
// compiled (int8 slots need int8 features), the rest as IQ = 2.
template <int CT, int KS, int KT, int IQ>
__device__ __attribute__((noinline)) void sweep_item(EncodeArgs &a, uint8_t *smem, int64_t qblock, const int32_t *truth,
                                                     SlotCount *res)
{
    if constexpr (IQ == 3 && dma_sweep_fits(CT, KS, KT)) {
        if (CT != C_I8 || a.x_type == X_INT8) {
            sweep_pass_dma<CT, KS, KT, 2, 2>(a, smem, qblock, truth, res);
            return;
        }
    }
    if constexpr (IQ >= 2 && sweep_qt2(CT, KS, KT)) {
        sweep_pass<CT, 2, KS, KT>(a, smem, qblock, truth, res);
    } else {
#pragma unroll 1
        for (int p = 0; p < (IQ == 1 ? 1 : 2); ++p) {
            if (p > 0)
                __syncthreads();    // the previous pass's last LDS reads are done
            sweep_pass<CT, 1, KS, KT>(a, smem, qblock + (int64_t)p * 32 * kWaves, truth, res);
        }
    }
}

template <int CT, int KS, int KT, int QT, int RT>
constexpr int dma_lds()
{
    if constexpr (dma_sweep_fits(CT, KS, KT))
        return Encoder<CT, 0, QT, KS, KT, M_CLASSIFY, 1, true, RT>::LDS;
    else
        return 0;
}

template <int FB, int KT, int IQ>
struct SweepLds {
    static constexpr int a = Encoder<C_I8, 0, 2, FB / 32, KT, M_CLASSIFY, 1>::LDS;
    static constexpr int b = Encoder<C_FP8, 0, 1, FB / 64, KT, M_CLASSIFY, 1>::LDS;
    static constexpr int c = Encoder<C_BF16, 0, 1, FB / 16, KT, M_CLASSIFY, 1>::LDS;
    static constexpr int d = Encoder<C_I8, 0, 1, FB / 32, KT, M_CLASSIFY, 1>::LDS;
    static constexpr int e = IQ == 3 ? dma_lds<C_I8, FB / 32, KT, 2, 2>() : 0;
    static constexpr int f = IQ == 3 ? dma_lds<C_FP8, FB / 64, KT, 2, 2>() : 0;
    static constexpr int ab = a > b ? a : b;
    static constexpr int cd = c > d ? c : d;
    static constexpr int ef = e > f ? e : f;
    static constexpr int abcd = ab > cd ? ab : cd;
    static constexpr int value = abcd > ef ? abcd : ef;
};

// The persistent kernel.  Each slot runs with its own work-item size (its
// configuration's tile id); the LDS holds the largest body of the bucket.
template <int FB, int KT>
__global__ __launch_bounds__(256) void k_sweep(EncodeArgs base, const int32_t *__restrict__ truth,
                                               uint8_t *__restrict__ ws, SweepLayout L, size_t table_bytes,
                                               int ncfg, int64_t ldp_conv)
{
    __shared__ __align__(16) uint8_t smem[SweepLds<FB, KT, 3>::value];
    __shared__ int item_s;
    const SlotDesc *desc = (const SlotDesc *)(ws + L.off_desc);
    const int32_t *order = (const int32_t *)(ws + L.off_order);
    const int32_t *items = (const int32_t *)(ws + L.off_items);
    SlotCount *cnt = (SlotCount *)(ws + L.off_count);
    const int total = items[ncfg];
    for (;;) {
        if (threadIdx.x == 0)
            item_s = (int)atomicAdd((uint32_t *)ws, 1u);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= total)
            break;
        // rank of the item: the last r with items[r] <= item
        int lo = 0, hi = ncfg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid] <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int slot = order[lo];
        const int tile = item - items[lo];
        const SlotDesc s = desc[slot];
        if (s.ct < 0)
            continue;
        const uint64_t t0 = wall_clock64();
        EncodeArgs a = base;
        a.s0 = s.s0;
        a.stride = s.stride;
        a.nd = s.nd;
        // the direct-staged E4M3 body reads the converted rows
        if (s.iq == 3 && s.ct == C_FP8 && dma_sweep_fits(C_FP8, FB / 64, KT)) {
            a.P = (const int8_t *)(ws + L.off_p8);
            a.ldp = ldp_conv;
        }
        a.ctab = (const int8_t *)(ws + L.off_regions + L.region * s.table);
        a.cpop = (const int32_t *)(ws + L.off_regions + L.region * s.table + table_bytes);
        const int64_t qblock = (int64_t)tile * (s.iq == 1 ? 1 : 2) * 32 * kWaves;
        SlotCount *res = &cnt[slot];
        if (s.ct == C_I8) {
            if (s.iq == 1)
                sweep_item<C_I8, FB / 32, KT, 1>(a, smem, qblock, truth, res);
            else if (s.iq == 2)
                sweep_item<C_I8, FB / 32, KT, 2>(a, smem, qblock, truth, res);
            else
                sweep_item<C_I8, FB / 32, KT, 3>(a, smem, qblock, truth, res);
        } else if (s.ct == C_FP8) {
            if (s.iq == 1)
                sweep_item<C_FP8, FB / 64, KT, 1>(a, smem, qblock, truth, res);
            else if (s.iq == 2)
                sweep_item<C_FP8, FB / 64, KT, 2>(a, smem, qblock, truth, res);
            else
                sweep_item<C_FP8, FB / 64, KT, 3>(a, smem, qblock, truth, res);
        } else {
            if (s.iq == 1)
                sweep_item<C_BF16, FB / 16, KT, 1>(a, smem, qblock, truth, res);
            else
                sweep_item<C_BF16, FB / 16, KT, 2>(a, smem, qblock, truth, res);
        }
        if (threadIdx.x == 0)
            atomicAdd((unsigned long long *)&res->ticks, (unsigned long long)(wall_clock64() - t0));
    }
}

template <int FB, int KT>
static hipError_t launch_sweep_kernel(const EncodeArgs &base, const SweepArgs &a, const SweepLayout &L,
                                      size_t table_bytes, hipStream_t st)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep<FB, KT>, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int grid = cus * per_cu;
    if (a.max_wg > 0 && a.max_wg < grid)
        grid = a.max_wg;
    hipLaunchKernelGGL((k_sweep<FB, KT>), dim3(grid), dim3(256), 0, st, base, a.truth, a.ws, L, table_bytes,
                       a.ncfg, (int64_t)L.ldp_conv);
    return hipGetLastError();
}

template <int FB>
static hipError_t launch_sweep_fb(const EncodeArgs &base, const SweepArgs &a, const SweepLayout &L,
                                  size_t table_bytes, hipStream_t st)
{
    if (sweep_kt(a.K) == 1)
        return launch_sweep_kernel<FB, 1>(base, a, L, table_bytes, st);
    return launch_sweep_kernel<FB, 4>(base, a, L, table_bytes, st);
}

hipError_t launch_sweep(const SweepArgs &a, hipStream_t st)
{
    const SweepLayout L(a.ncfg, a.F, a.D, a.K);
    const int KT = sweep_kt(a.K);
    const size_t table_bytes = sweep_table_bytes(a.D, a.K);
    // ---- host setup: slot descriptors, order, work items, distinct sets
    std::vector<uint8_t> blob(L.off_regions, 0);
    SlotDesc *desc = (SlotDesc *)(blob.data() + L.off_desc);
    int32_t *order = (int32_t *)(blob.data() + L.off_order);
    int32_t *items = (int32_t *)(blob.data() + L.off_items);
    SlotCount *cnt = (SlotCount *)(blob.data() + L.off_count);
    TableDesc *tabs = (TableDesc *)(blob.data() + L.off_tabs);
    std::vector<int64_t> cost(a.ncfg);
    std::map<std::tuple<int, int, int>, int> seen;
    // shared configurations: chains (compute type, start, stride) -> end ->
    // end counter, and the dimension range [lo, hi) of each compute type
    std::map<std::tuple<int, int, int>, std::map<int, int>> chains;
    std::map<int, std::pair<int, int>> ranges;
    int nslots = 0;
    bool direct = false;
    for (int i = 0; i < a.ncfg; ++i) {
        const hdc_config c = a.cfgs[i];
        SlotDesc s;
        memset(&s, 0, sizeof s);
        s.ct = c.dtype == HDC_INT8 ? C_I8 : c.dtype == HDC_BF16 ? C_BF16 : c.dtype == HDC_FP8_E4M3 ? C_FP8 : -1;
        const bool ok = s.ct >= 0 && c.stride >= 1 && c.start >= 0 && c.d_trunc > c.start && c.d_trunc <= a.D;
        if (!ok)
            s.ct = -1;
        s.s0 = ok ? c.start : 0;
        s.stride = ok ? c.stride : 1;
        s.nd = ok ? (c.d_trunc - c.start + c.stride - 1) / c.stride : 0;
        // built-in work items: 256 queries
        s.iq = c.tile_id == SV_ITEM128 ? 1 : c.tile_id == SV_ITEM256_DMA ? 3 : c.tile_id == SV_SHARED ? SV_SHARED : 2;
        s.tiles = ok && s.iq != SV_SHARED ? (int32_t)((a.n + (s.iq == 1 ? 127 : 255)) / (s.iq == 1 ? 128 : 256)) : 0;
        if (ok && s.iq == SV_SHARED) {
            // its end counter: one per distinct (encoding, start, stride,
            // end).  Integer features (|x| <= 255) and +-1 rows are exact in
            // bf16 and so are the sums (|y| < 2^24) in its fp32 accumulator:
            // the bf16 encoding is the exact integer encoding, the int8 one.
            const int rct = s.ct == C_BF16 ? C_I8 : s.ct;
            const int end = s.s0 + (s.nd - 1) * s.stride + 1;
            auto &ch = chains[std::make_tuple(rct, s.s0, s.stride)];
            auto it = ch.find(end);
            if (it == ch.end())
                it = ch.emplace(end, nslots++).first;
            s.table = it->second;
            auto rg_it = ranges.find(rct);
            if (rg_it == ranges.end())
                rg_it = ranges.emplace(rct, std::make_pair(a.D, 0)).first;
            auto &rg = rg_it->second;
            if (rg.first > s.s0 / 64 * 64)
                rg.first = s.s0 / 64 * 64;
            if (rg.second < end)
                rg.second = end;
        } else if (ok) {
            const auto key = std::make_tuple(s.s0, s.stride, s.nd);
            auto it = seen.find(key);
            if (it == seen.end()) {
                const int t = (int)seen.size();
                it = seen.emplace(key, t).first;
                tabs[t] = TableDesc{s.s0, s.stride, s.nd, 0};
            }
            s.table = it->second;
            direct |= s.iq == 3 && s.ct == C_FP8;
        }
        desc[i] = s;
        cost[i] = (int64_t)s.nd * (s.ct == C_BF16 ? 2 : 1);
        cnt[i].correct = 0;
        cnt[i].n = ok ? (int32_t)a.n : 0;
        cnt[i].ticks = 0;
        order[i] = i;
    }
    std::stable_sort(order, order + a.ncfg, [&](int x, int y) { return cost[x] > cost[y]; });
    int32_t run = 0;
    for (int r = 0; r < a.ncfg; ++r) {
        items[r] = run;
        run += desc[order[r]].tiles;
    }
    items[a.ncfg] = run;
    const int ntab = (int)seen.size();
    // shared search items: each chain's ends in groups of kShEnds, longest
    // word range first; one encoding region per compute type
    std::map<int, int> reg_of;
    std::vector<int> reg_ct;
    for (const auto &r : ranges) {
        reg_of[r.first] = (int)reg_ct.size();
        reg_ct.push_back(r.first);
    }
    std::vector<ShItem> sh;
    for (const auto &ch : chains) {
        const int ct = std::get<0>(ch.first), s0 = std::get<1>(ch.first), stride = std::get<2>(ch.first);
        std::vector<std::pair<int, int>> ends(ch.second.begin(), ch.second.end());
        for (size_t g = 0; g < ends.size(); g += kShEnds) {
            ShItem t;
            memset(&t, 0, sizeof t);
            t.reg = reg_of[ct];
            t.s0 = s0;
            t.stride = stride;
            t.wlo = ranges[ct].first / 64;
            t.nend = (int)(ends.size() - g < (size_t)kShEnds ? ends.size() - g : kShEnds);
            for (int x = 0; x < t.nend; ++x) {
                t.end[x] = ends[g + x].first;
                t.slot[x] = ends[g + x].second;
            }
            t.a0 = s0 / 64;
            t.a1 = (t.end[t.nend - 1] - 1) / 64 + 1;
            sh.push_back(t);
        }
    }
    std::stable_sort(sh.begin(), sh.end(), [](const ShItem &x, const ShItem &y) { return x.a1 - x.a0 > y.a1 - y.a0; });
    if (!sh.empty())
        memcpy(blob.data() + L.off_sh, sh.data(), sh.size() * sizeof(ShItem));
    // the queue counter (offset 0) goes up as 0 with the rest
    hipError_t e = hipMemcpyAsync(a.ws, blob.data(), blob.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess)
        return e;
    if (ntab > 0) {
        const int64_t per_slot = table_chunks(a.D) * KT * 64;
        const unsigned gx = (unsigned)((per_slot + 255) / 256 < 1024 ? (per_slot + 255) / 256 : 1024);
        hipLaunchKernelGGL(k_sweep_tables, dim3(gx, ntab), dim3(256), 0, st, a.C, a.K, a.ldc, a.ws, L, KT,
                           per_slot);
        hipLaunchKernelGGL(k_sweep_popc, dim3(KT * 32, ntab), dim3(256), 0, st, a.C, a.K, a.ldc, a.ws, L,
                           table_bytes);
    }
    if (direct) {
        const int64_t total = (int64_t)a.D * (int64_t)L.ldp_conv;
        const int64_t g = (total + 255) / 256;
        hipLaunchKernelGGL(k_sweep_convert, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, st, a.P, a.ldp, a.D,
                           a.F, a.ws, L);
    }
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    EncodeArgs base;
    memset(&base, 0, sizeof base);
    base.X = a.X;
    base.x_type = a.x_type;
    base.n = a.n;
    base.F = a.F;
    base.ldx = a.ldx;
    base.P = a.P;
    base.ldp = a.ldp;
    base.K = a.K;
    if (run > 0) {
        if (a.F <= 128) e = launch_sweep_fb<128>(base, a, L, table_bytes, st);
        else if (a.F <= 256) e = launch_sweep_fb<256>(base, a, L, table_bytes, st);
        else if (a.F <= 512) e = launch_sweep_fb<512>(base, a, L, table_bytes, st);
        else if (a.F <= 640) e = launch_sweep_fb<640>(base, a, L, table_bytes, st);
        else if (a.F <= 832) e = launch_sweep_fb<832>(base, a, L, table_bytes, st);
        else e = launch_sweep_fb<1024>(base, a, L, table_bytes, st);
        if (e != hipSuccess)
            return e;
    }
    // shared configurations, kShQueries queries per pass: encode the range
    // of each compute type, then one search launch over every item
    for (int64_t q0 = 0; !sh.empty() && q0 < a.n; q0 += kShQueries) {
        const int nq = (int)(a.n - q0 < kShQueries ? a.n - q0 : kShQueries);
        for (size_t r = 0; r < reg_ct.size(); ++r) {
            EncodeArgs ea = base;
            ea.X = (const int8_t *)a.X + q0 * a.ldx;
            ea.n = nq;
            ea.s0 = ranges[reg_ct[r]].first;
            ea.stride = 1;
            ea.nd = ranges[reg_ct[r]].second - ea.s0;
            ea.H32 = (uint32_t *)(a.ws + L.off_h + L.hreg * r);
            ea.ldh32 = 2 * (int64_t)L.wd;
            ea.max_split = 1 << 30;
            e = launch_encode(ea, reg_ct[r], M_ENCODE, Tile{0}, st);
            if (e != hipSuccess)
                return e;
        }
        const dim3 grid((unsigned)((nq + 63) / 64), (unsigned)sh.size());
        // eight waves per query block, K / 8 classes each (rounded up to 4, 8, 16)
        if (a.K <= 32)
            hipLaunchKernelGGL((k_sweep_shared<4, 8>), grid, dim3(512), 0, st, a.C, a.K, a.ldc, a.truth + q0, nq,
                               a.ws, L);
        else if (a.K <= 64)
            hipLaunchKernelGGL((k_sweep_shared<8, 8>), grid, dim3(512), 0, st, a.C, a.K, a.ldc, a.truth + q0, nq,
                               a.ws, L);
        else
            hipLaunchKernelGGL((k_sweep_shared<16, 8>), grid, dim3(512), 0, st, a.C, a.K, a.ldc, a.truth + q0, nq,
                               a.ws, L);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    // results: ticks -> microseconds of the device wall clock, then down to
    // the caller's host array (from pinned memory the copy stays
    // asynchronous; into pageable memory the runtime completes it first)
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) !=
                                                hipSuccess || khz <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sweep_results, dim3((unsigned)((a.ncfg + 255) / 256)), dim3(256), 0, st, a.ncfg, a.ws, L,
                       1000.0 / (double)khz);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return hipMemcpyAsync(a.out, a.ws + L.off_res, (size_t)a.ncfg * sizeof(hdc_config_result),
                          hipMemcpyDeviceToHost, st);
}

}  // namespace hdc
