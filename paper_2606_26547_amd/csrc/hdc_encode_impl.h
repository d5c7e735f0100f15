// Kernel entry points and launch dispatch of the encoder for one compute
// type.  Each hdc_encode_<type>.hip defines HDC_CT and includes this file,
// so the instantiations of the four compute types compile in parallel.
#pragma once

#include "hdc_encoder.h"

namespace hdc {

// Grid: query blocks, or (dimension split, query block) when the launch
// splits its dimensions (a.nsplit = Z > 1).  Split z of Z takes the whole
// 64-dimension words [z * per, (z + 1) * per) of the dimension list: its
// projection rows, its half-words of the packed output and its part of the
// class operand.  Workgroups are dealt to the XCDs in turn by linear id, so
// with the split index fastest each XCD's L2 holds the projection rows of
// its splits only, not all of them.  In classify mode every split adds its
// own part of the class sums, so a split launch writes them to
// part[z][n][K] and k_split_argmin finishes.
template <int CT, int XF, int QT, int KS, int KT, int MODE, bool DMA, int RT>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(Encoder<CT, XF, QT, KS, KT, MODE, 0, DMA, RT>::WAVES)))
void k_encode(EncodeArgs a)
{
    typedef Encoder<CT, XF, QT, KS, KT, MODE, 0, DMA, RT> E;
    __shared__ __align__(16) uint8_t smem[E::LDS];
    const int Z = a.nsplit;
    const int z = Z > 1 ? (int)blockIdx.x : 0;
    const int64_t qblock = (int64_t)(Z > 1 ? blockIdx.y : blockIdx.x) * E::QPB;
    if (Z > 1) {
        const int per = split_units(a.nd, Z);
        const int d0 = 64 * z * per;                    // first dimension (list index) of the split
        const int nd = a.nd - d0 < 64 * per ? a.nd - d0 : 64 * per;
        a.s0 += d0 * a.stride;
        a.nd = nd;
        if constexpr (MODE == M_ENCODE)
            a.H32 += d0 / 32;
        else
            a.ctab += (int64_t)(d0 / 32) * KT * 1024;
    }
    v16i dacc[KT][QT];
    E::run(a, smem, qblock, dacc);
    if constexpr (MODE == M_CLASSIFY) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (Z > 1) {
            const int g = lane >> 5;
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) {
                const int64_t q = qblock + (int64_t)wave * E::QPW + qt * 32 + (lane & 31);
                if (q >= a.n)
                    continue;
#pragma unroll
                for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int k = kt * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
                        if (k < a.K)
                            a.part[((int64_t)z * a.n + q) * a.K + k] = dacc[kt][qt][v];
                    }
            }
            return;
        }
        int32_t lab[QT];
        E::finish(a, qblock, dacc, lab);
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            const int64_t q = qblock + (int64_t)wave * E::QPW + qt * 32 + (lane & 31);
            if (lane < 32 && q < a.n)
                a.labels[q] = lab[qt];
        }
    }
}

// Distances and argmin of a split classify launch: one wave per query,
// lane k (and k + 64) sums class k's partials over the splits, dist_k =
// popc_k - sum; the first smallest distance wins, as in Encoder::finish.
static __global__ __launch_bounds__(256) void k_split_argmin(EncodeArgs a, int Z)
{
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= a.n)
        return;
    int bd = 0x7fffffff, bk = 0;
    for (int k0 = 0; k0 < a.K; k0 += 64) {
        const int k = k0 + lane;
        const bool kv = k < a.K;
        int s = 0;
        if (kv) {
            const int32_t *p = a.part + q * a.K + k;
            const int64_t zs = a.n * a.K;
#pragma unroll 8
            for (int z = 0; z < Z; ++z)
                s += p[z * zs];
        }
        const int d = kv ? a.cpop[k] - s : 0x7fffffff;
        if (kv && a.dists)
            a.dists[q * a.K + k] = d;
        if (d < bd) {
            bd = d;
            bk = k;
        }
    }
    // first minimum across the lanes (lower class index on ties)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const int od = __shfl_xor(bd, o), ok = __shfl_xor(bk, o);
        if (od < bd || (od == bd && ok < bk)) {
            bd = od;
            bk = ok;
        }
    }
    if (lane == 0)
        a.labels[q] = bk;
}

template <int CT, int XF, int QT, int KS, int KT, int MODE, bool DMA = false, int RT = 1>
static hipError_t launch_one(const EncodeArgs &a, hipStream_t st)
{
    typedef Encoder<CT, XF, QT, KS, KT, MODE, 0, DMA, RT> E;
    const int64_t blocks = (a.n + E::QPB - 1) / E::QPB;
    // resident workgroups: one per CU per wave per SIMD the kernel is built for
    const int Z = split_count(blocks, a.nd, a.max_split, 256 * E::WAVES);
    EncodeArgs b = a;
    b.nsplit = Z;
    const dim3 grid = Z > 1 ? dim3((unsigned)Z, (unsigned)blocks) : dim3((unsigned)blocks);
    hipLaunchKernelGGL((k_encode<CT, XF, QT, KS, KT, MODE, DMA, RT>), grid, dim3(256), 0, st, b);
    if (MODE == M_CLASSIFY && Z > 1)
        hipLaunchKernelGGL(k_split_argmin, dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0, st, a, Z);
    return hipGetLastError();
}

// int8 features on the int8 path stage the projection straight into LDS.
// Where the registers allow (big_tile), each wave (one per SIMD) multiplies
// two query tiles by two row tiles per chunk: four independent accumulator
// chains, each projection fragment read from LDS feeds two MFMAs, and a
// barrier every 80 MFMAs; the classifier can also take three row tiles per
// chunk (TV_DMA_2X3: a barrier every 120 MFMAs, two stages).  Otherwise (or
// when the tile table asks for it) one tile of each, two waves per SIMD.
template <int KS, int KT, int MODE>
static hipError_t launch_dma(const EncodeArgs &a, int variant, hipStream_t st)
{
    if constexpr (MODE == M_CLASSIFY && big3_tile(KS, KT)) {
        // 96-dimension chunks: a dimension split would end inside a chunk
        // and read the next split's class tiles, so this shape never splits;
        // a batch the 2x2 shape would split (too few query blocks to fill
        // the device) runs on that shape instead
        if (variant == TV_DMA_2X3) {
            typedef Encoder<C_I8, 0, 2, KS, KT, MODE, 0, true, 2> E2;
            const int64_t blocks = (a.n + E2::QPB - 1) / E2::QPB;
            if (split_count(blocks, a.nd, a.max_split, 256 * E2::WAVES) == 1) {
                EncodeArgs b = a;
                b.max_split = 1;
                return launch_one<C_I8, 0, 2, KS, KT, MODE, true, 3>(b, st);
            }
        }
    }
    if (a.poff && (!shift_tile(KS, KT) || variant == TV_DMA_1X1))
        return hipErrorInvalidValue;   // the shifted projection: shift_tile shapes only
    if constexpr (big_tile(KS, KT)) {
        if (variant != TV_DMA_1X1)
            return launch_one<C_I8, 0, 2, KS, KT, MODE, true, 2>(a, st);
    }
    return launch_one<C_I8, 0, 1, KS, KT, MODE, true, 1>(a, st);
}

// One feature-width bucket: the tile variant picks direct or register
// staging and the query tiles per wave; 0 is the built-in rule (direct
// staging for int8 features on the int8 path, else as many query tiles as
// fit).
template <int CT, int XF, int KS>
static hipError_t launch_bucket(const EncodeArgs &a, int mode, Tile tile, hipStream_t st)
{
    const int v = tile.variant;
    if constexpr (CT == C_I8 && XF == 0) {
        const bool dma = a.x_type == X_INT8 && (v == TV_AUTO || v == TV_DMA_2X2 || v == TV_DMA_1X1 || v == TV_DMA_2X3);
        if (a.poff && !dma)   // the shifted projection runs on direct staging only
            return hipErrorInvalidValue;
        if (dma) {
            if (mode == M_ENCODE)
                return launch_dma<KS, 1, M_ENCODE>(a, v, st);
            const int kt = class_tiles(a.K);
            if (kt == 1)
                return launch_dma<KS, 1, M_CLASSIFY>(a, v, st);
            if (kt == 2)
                return launch_dma<KS, 2, M_CLASSIFY>(a, v, st);
            return launch_dma<KS, 4, M_CLASSIFY>(a, v, st);
        }
    }
    if constexpr (CT == C_FP8 && XF == 0) {
        // E4M3 on the shifted projection (rows of E4M3 bytes 0 / 2.0, poff
        // set): the direct-staged 2x2 shape, shift8_tile widths only
        if (a.poff) {
            if (v != TV_AUTO && v != TV_DMA_2X2)
                return hipErrorInvalidValue;
            if constexpr (shift8_tile(KS, 2)) {
                if (mode == M_ENCODE)
                    return launch_one<C_FP8, 0, 1, KS, 1, M_ENCODE, true, 1>(a, st);
                const int kt = class_tiles(a.K);
                if (kt == 1)
                    return launch_one<C_FP8, 0, 1, KS, 1, M_CLASSIFY, true, 1>(a, st);
                if (kt == 2)
                    return launch_one<C_FP8, 0, 1, KS, 2, M_CLASSIFY, true, 1>(a, st);
            }
            return hipErrorInvalidValue;
        }
    }
    if (a.poff)
        return hipErrorInvalidValue;
    constexpr int QM = qt2_fits(CT, KS) ? 2 : 1;
    const int qt = (v == TV_REG_QT1 || QM == 1) ? 1 : 2;
    if (mode == M_ENCODE) {
        if (qt == 2)
            return launch_one<CT, XF, QM, KS, 1, M_ENCODE>(a, st);
        return launch_one<CT, XF, 1, KS, 1, M_ENCODE>(a, st);
    }
    const int kt = class_tiles(a.K);
    if (kt == 1) {
        if (qt == 2)
            return launch_one<CT, XF, QM, KS, 1, M_CLASSIFY>(a, st);
        return launch_one<CT, XF, 1, KS, 1, M_CLASSIFY>(a, st);
    }
    if (kt == 2) {
        if (qt == 2)
            return launch_one<CT, XF, QM, KS, 2, M_CLASSIFY>(a, st);
        return launch_one<CT, XF, 1, KS, 2, M_CLASSIFY>(a, st);
    }
    return launch_one<CT, XF, 1, KS, 4, M_CLASSIFY>(a, st);
}

// Feature-count buckets: the smallest compiled width >= F is used.
template <int CT>
static hipError_t launch_encode_ct(const EncodeArgs &a, int mode, Tile tile, hipStream_t st)
{
    constexpr int KSTEP = Tr<CT>::KSTEP;
    const int F = a.F;
    if (a.x_type == X_FP32) {
        if constexpr (CT == C_I8 || CT == C_FP8S) {
            return hipErrorInvalidValue;
        } else {
            if (F <= 64) return launch_bucket<CT, 1, 64 / KSTEP>(a, mode, tile, st);
            if (F <= 128) return launch_bucket<CT, 1, 128 / KSTEP>(a, mode, tile, st);
            if (F <= 256) return launch_bucket<CT, 1, 256 / KSTEP>(a, mode, tile, st);
            return hipErrorInvalidValue;
        }
    }
    if constexpr (CT == C_F32) {
        return hipErrorInvalidValue;
    } else {
        constexpr int K1 = 64 / KSTEP > 0 ? 64 / KSTEP : 1;
        if (F <= 64) return launch_bucket<CT, 0, K1>(a, mode, tile, st);
        if (F <= 128) return launch_bucket<CT, 0, 128 / KSTEP>(a, mode, tile, st);
        if (F <= 192) return launch_bucket<CT, 0, 192 / KSTEP>(a, mode, tile, st);
        if (F <= 256) return launch_bucket<CT, 0, 256 / KSTEP>(a, mode, tile, st);
        if (F <= 320) return launch_bucket<CT, 0, 320 / KSTEP>(a, mode, tile, st);
        if (F <= 384) return launch_bucket<CT, 0, 384 / KSTEP>(a, mode, tile, st);
        if (F <= 512) return launch_bucket<CT, 0, 512 / KSTEP>(a, mode, tile, st);
        if (F <= 640) return launch_bucket<CT, 0, 640 / KSTEP>(a, mode, tile, st);
        if (F <= 832) return launch_bucket<CT, 0, 832 / KSTEP>(a, mode, tile, st);
        if (F <= 1024) return launch_bucket<CT, 0, 1024 / KSTEP>(a, mode, tile, st);
        return hipErrorInvalidValue;
    }
}

}  // namespace hdc
