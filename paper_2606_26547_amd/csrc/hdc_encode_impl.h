// Kernel entry points and launch dispatch of the encoder for one compute
// type.  Each hdc_encode_<type>.hip defines HDC_CT and includes this file,
// so the instantiations of the four compute types compile in parallel.
#pragma once

#include "hdc_encoder.h"

namespace hdc {

template <int CT, int XF, int QT, int KS, int KT, int MODE, bool DMA, int RT>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(Encoder<CT, XF, QT, KS, KT, MODE, 0, DMA, RT>::WAVES)))
void k_encode(EncodeArgs a)
{
    typedef Encoder<CT, XF, QT, KS, KT, MODE, 0, DMA, RT> E;
    __shared__ __align__(16) uint8_t smem[E::LDS];
    const int64_t qblock = (int64_t)blockIdx.x * E::QPB;
    v16i dacc[KT][QT];
    E::run(a, smem, qblock, dacc);
    if constexpr (MODE == M_CLASSIFY) {
        int32_t lab[QT];
        E::finish(a, qblock, dacc, lab);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
            const int64_t q = qblock + (int64_t)wave * E::QPW + qt * 32 + (lane & 31);
            if (lane < 32 && q < a.n)
                a.labels[q] = lab[qt];
        }
    }
}

template <int CT, int XF, int QT, int KS, int KT, int MODE, bool DMA = false, int RT = 1>
static hipError_t launch_one(const EncodeArgs &a, hipStream_t st)
{
    typedef Encoder<CT, XF, QT, KS, KT, MODE, 0, DMA, RT> E;
    const int64_t blocks = (a.n + E::QPB - 1) / E::QPB;
    hipLaunchKernelGGL((k_encode<CT, XF, QT, KS, KT, MODE, DMA, RT>), dim3((unsigned)blocks), dim3(256), 0, st,
                       a);
    return hipGetLastError();
}

// int8 features on the int8 path stage the projection straight into LDS.
// Where the registers allow (big_tile), each wave (one per SIMD) multiplies
// two query tiles by two row tiles per chunk: four independent accumulator
// chains, each projection fragment read from LDS feeds two MFMAs, and a
// barrier every 80 MFMAs.  Otherwise (or when the tile table asks for it)
// one tile of each, two waves per SIMD.
template <int KS, int KT, int MODE>
static hipError_t launch_dma(const EncodeArgs &a, int variant, hipStream_t st)
{
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
        if (a.x_type == X_INT8 && (v == TV_AUTO || v == TV_DMA_2X2 || v == TV_DMA_1X1)) {
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
