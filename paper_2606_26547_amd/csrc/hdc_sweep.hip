// hdc_eval_configs: one persistent launch that classifies the same queries
// under many approximation configurations (the inner loop of the tuning
// system: run each candidate, read back its accuracy and time).
//
// Workspace layout (all offsets 256-byte aligned):
//   [0]            queue counter (uint32) and item count
//   [256]          slot descriptors, ncfg x SlotDesc
//   [..]           slot order (longest first), ncfg x int32
//   [..]           per-slot class operand regions of fixed size
//                  (chunks(D) * KT KiB table + 128 int32 popcounts)
// Work item i = (slot order[i / tiles], query tile i % tiles); a workgroup
// takes items from the queue until it is exhausted, so every workgroup
// reaches the exit whatever the grid size.
#include <string.h>

#include "hdc_encoder.h"

namespace hdc {

struct SlotDesc {
    int32_t s0, stride, nd, ct;   // ct < 0: invalid configuration (no work)
    int64_t cost;
};


inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Class tiles compiled into the sweep kernel: 1 (K <= 32) or 4 (K <= 128).
// A slot's table holds whole pairs of 32-dimension chunks (the direct-staged
// 2x2 body reads them in pairs; the pad chunk is zero).
inline size_t sweep_table_bytes(int D, int K) { return (size_t)table_chunks(D) * sweep_kt(K) * 1024; }

struct SweepLayout {
    size_t off_desc, off_order, off_regions, region, total;
    SweepLayout(int ncfg, int D, int K)
    {
        off_desc = 256;
        off_order = align256(off_desc + (size_t)ncfg * sizeof(SlotDesc));
        off_regions = align256(off_order + (size_t)ncfg * 4);
        region = align256(sweep_table_bytes(D, K) + 128 * 4);
        total = off_regions + region * (size_t)ncfg;
    }
};

size_t sweep_workspace_bytes(int32_t ncfg, int32_t D, int32_t K)
{
    if (ncfg <= 0 || D <= 0 || K <= 0 || K > kMaxK)
        return 0;
    return SweepLayout(ncfg, D, K).total;
}

// Validate configurations, zero the results and order the slots by
// decreasing cost (dimensions x compute cost); ties keep slot order.
__global__ __launch_bounds__(1024) void k_sweep_setup(const hdc_config *__restrict__ cfgs, int ncfg, int D,
                                                      int64_t n, uint8_t *__restrict__ ws,
                                                      hdc_config_result *__restrict__ out, size_t off_desc,
                                                      size_t off_order)
{
    SlotDesc *desc = (SlotDesc *)(ws + off_desc);
    int32_t *order = (int32_t *)(ws + off_order);
    for (int i = threadIdx.x; i < ncfg; i += blockDim.x) {
        const hdc_config c = cfgs[i];
        SlotDesc s;
        s.s0 = c.start;
        s.stride = c.stride;
        s.ct = c.dtype == HDC_INT8 ? C_I8 : c.dtype == HDC_BF16 ? C_BF16 : c.dtype == HDC_FP8_E4M3 ? C_FP8 : -1;
        const bool ok = s.ct >= 0 && c.stride >= 1 && c.start >= 0 && c.d_trunc > c.start && c.d_trunc <= D;
        if (!ok)
            s.ct = -1;
        s.nd = ok ? (c.d_trunc - c.start + c.stride - 1) / c.stride : 0;
        s.cost = (int64_t)s.nd * (s.ct == C_BF16 ? 2 : 1);
        desc[i] = s;
        out[i].correct = 0;
        out[i].n = ok ? (int32_t)n : 0;
        out[i].ticks = 0;
    }
    if (threadIdx.x == 0)
        ((uint32_t *)ws)[0] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < ncfg; i += blockDim.x) {
        const int64_t ci = desc[i].cost;
        int rank = 0;
        for (int j = 0; j < ncfg; ++j) {
            const int64_t cj = desc[j].cost;
            rank += (cj > ci) || (cj == ci && j < i);
        }
        order[rank] = i;
    }
}

// Class operand tables of every slot (same layout as hdc_classify's).
__global__ __launch_bounds__(256) void k_sweep_tables(const uint64_t *__restrict__ C, int K, int64_t ldc,
                                                      uint8_t *__restrict__ ws, size_t off_desc,
                                                      size_t off_regions, size_t region, int KT, int64_t per_slot)
{
    const int slot = blockIdx.y;
    const SlotDesc s = ((const SlotDesc *)(ws + off_desc))[slot];
    int8_t *tab = (int8_t *)(ws + off_regions + region * slot);
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
                                                    uint8_t *__restrict__ ws, size_t off_desc, size_t off_regions,
                                                    size_t region, size_t table_bytes)
{
    __shared__ int part[256];
    const int slot = blockIdx.y, k = blockIdx.x;
    const SlotDesc s = ((const SlotDesc *)(ws + off_desc))[slot];
    int32_t *popc = (int32_t *)(ws + off_regions + region * slot + table_bytes);
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

// One encoder pass of QT query tiles per wave over the queries from qblock,
// adding the correct labels to the slot's count.
template <int CT, int QT, int KS, int KT>
__device__ __forceinline__ void sweep_pass(EncodeArgs &a, uint8_t *smem, int64_t qblock, const int32_t *truth,
                                           hdc_config_result *res)
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

// The fused classifier's direct-staged 2x2 body on one 256-query item
// (int8 features on the int8 path).
template <int KS, int KT>
__device__ __forceinline__ void sweep_pass_dma(EncodeArgs &a, uint8_t *smem, int64_t qblock, const int32_t *truth,
                                               hdc_config_result *res)
{
    typedef Encoder<C_I8, 0, 2, KS, KT, M_CLASSIFY, 1, true, 2> E;
    v16i dacc[KT][2];
    E::run(a, smem, qblock, dacc);
    int32_t lab[2];
    E::finish(a, qblock, dacc, lab);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int qt = 0; qt < 2; ++qt) {
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
// run two passes; IQ = 3 runs int8-feature int8 slots on the direct-staged
// 2x2 body instead (where it is compiled), the rest as IQ = 2.
template <int CT, int KS, int KT, int IQ>
__device__ __attribute__((noinline)) void sweep_item(EncodeArgs &a, uint8_t *smem, int64_t qblock, const int32_t *truth,
                                                     hdc_config_result *res)
{
    if constexpr (IQ == 3 && CT == C_I8 && big_tile(KS, KT)) {
        if (a.x_type == X_INT8) {
            sweep_pass_dma<KS, KT>(a, smem, qblock, truth, res);
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

template <int FB, int KT, int IQ>
struct SweepLds {
    static constexpr int a = Encoder<C_I8, 0, 2, FB / 32, KT, M_CLASSIFY, 1>::LDS;
    static constexpr int b = Encoder<C_FP8, 0, 1, FB / 64, KT, M_CLASSIFY, 1>::LDS;
    static constexpr int c = Encoder<C_BF16, 0, 1, FB / 16, KT, M_CLASSIFY, 1>::LDS;
    static constexpr int d = Encoder<C_I8, 0, 1, FB / 32, KT, M_CLASSIFY, 1>::LDS;
    static constexpr int e = (IQ == 3 && big_tile(FB / 32, KT))
                                 ? Encoder<C_I8, 0, 2, FB / 32, KT, M_CLASSIFY, 1, true, 2>::LDS : 0;
    static constexpr int ab = a > b ? a : b;
    static constexpr int cd = c > d ? c : d;
    static constexpr int abcd = ab > cd ? ab : cd;
    static constexpr int value = abcd > e ? abcd : e;
};

template <int FB, int KT, int IQ>
__global__ __launch_bounds__(256) void k_sweep(EncodeArgs base, const int32_t *__restrict__ truth,
                                               uint8_t *__restrict__ ws, hdc_config_result *__restrict__ out,
                                               size_t off_desc, size_t off_order, size_t off_regions,
                                               size_t region, size_t table_bytes, int ncfg, int tiles)
{
    __shared__ __align__(16) uint8_t smem[SweepLds<FB, KT, IQ>::value];
    __shared__ int item_s;
    const SlotDesc *desc = (const SlotDesc *)(ws + off_desc);
    const int32_t *order = (const int32_t *)(ws + off_order);
    const int total = ncfg * tiles;
    for (;;) {
        if (threadIdx.x == 0)
            item_s = (int)atomicAdd((uint32_t *)ws, 1u);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= total)
            break;
        const int slot = order[item / tiles];
        const int tile = item % tiles;
        const SlotDesc s = desc[slot];
        if (s.ct < 0)
            continue;
        const uint64_t t0 = wall_clock64();
        EncodeArgs a = base;
        a.s0 = s.s0;
        a.stride = s.stride;
        a.nd = s.nd;
        a.ctab = (const int8_t *)(ws + off_regions + region * slot);
        a.cpop = (const int32_t *)(ws + off_regions + region * slot + table_bytes);
        const int64_t qblock = (int64_t)tile * (IQ == 1 ? 1 : 2) * 32 * kWaves;
        if (s.ct == C_I8)
            sweep_item<C_I8, FB / 32, KT, IQ>(a, smem, qblock, truth, &out[slot]);
        else if (s.ct == C_FP8)
            sweep_item<C_FP8, FB / 64, KT, IQ>(a, smem, qblock, truth, &out[slot]);
        else
            sweep_item<C_BF16, FB / 16, KT, IQ>(a, smem, qblock, truth, &out[slot]);
        if (threadIdx.x == 0)
            atomicAdd((unsigned long long *)&out[slot].ticks, (unsigned long long)(wall_clock64() - t0));
    }
}

template <int FB, int KT, int IQ>
static hipError_t launch_sweep_kernel(const EncodeArgs &base, const SweepArgs &a, const SweepLayout &L,
                                      size_t table_bytes, hipStream_t st)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep<FB, KT, IQ>, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int grid = cus * per_cu;
    if (a.max_wg > 0 && a.max_wg < grid)
        grid = a.max_wg;
    constexpr int QI = (IQ == 1 ? 1 : 2) * 32 * kWaves;   // queries per item
    const int tiles = (int)((a.n + QI - 1) / QI);
    hipLaunchKernelGGL((k_sweep<FB, KT, IQ>), dim3(grid), dim3(256), 0, st, base, a.truth, a.ws, a.out, L.off_desc,
                       L.off_order, L.off_regions, L.region, table_bytes, a.ncfg, tiles);
    return hipGetLastError();
}

// Work-item size from the tile table (0: the built-in 128 queries).
template <int FB>
static hipError_t launch_sweep_fb(const EncodeArgs &base, const SweepArgs &a, const SweepLayout &L,
                                  size_t table_bytes, hipStream_t st)
{
    const int v = get_tile(KK_SWEEP, a.x_type, C_I8, a.F, a.K);
    if (sweep_kt(a.K) == 1) {
        if constexpr (big_tile(FB / 32, 1)) {
            if (v == SV_ITEM256_DMA)
                return launch_sweep_kernel<FB, 1, 3>(base, a, L, table_bytes, st);
        }
        return v == SV_ITEM256 ? launch_sweep_kernel<FB, 1, 2>(base, a, L, table_bytes, st)
                               : launch_sweep_kernel<FB, 1, 1>(base, a, L, table_bytes, st);
    }
    return v == SV_ITEM256 ? launch_sweep_kernel<FB, 4, 2>(base, a, L, table_bytes, st)
                           : launch_sweep_kernel<FB, 4, 1>(base, a, L, table_bytes, st);
}

hipError_t launch_sweep(const SweepArgs &a, hipStream_t st)
{
    const SweepLayout L(a.ncfg, a.D, a.K);
    const int KT = sweep_kt(a.K);
    const size_t table_bytes = sweep_table_bytes(a.D, a.K);
    hipLaunchKernelGGL(k_sweep_setup, dim3(1), dim3(1024), 0, st, a.cfgs, a.ncfg, a.D, a.n, a.ws, a.out,
                       L.off_desc, L.off_order);
    const int64_t per_slot = table_chunks(a.D) * KT * 64;
    const unsigned gx = (unsigned)((per_slot + 255) / 256 < 1024 ? (per_slot + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_sweep_tables, dim3(gx, a.ncfg), dim3(256), 0, st, a.C, a.K, a.ldc, a.ws, L.off_desc,
                       L.off_regions, L.region, KT, per_slot);
    hipLaunchKernelGGL(k_sweep_popc, dim3(KT * 32, a.ncfg), dim3(256), 0, st, a.C, a.K, a.ldc, a.ws, L.off_desc,
                       L.off_regions, L.region, table_bytes);
    hipError_t e = hipGetLastError();
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
    if (a.F <= 128) return launch_sweep_fb<128>(base, a, L, table_bytes, st);
    if (a.F <= 256) return launch_sweep_fb<256>(base, a, L, table_bytes, st);
    if (a.F <= 512) return launch_sweep_fb<512>(base, a, L, table_bytes, st);
    if (a.F <= 640) return launch_sweep_fb<640>(base, a, L, table_bytes, st);
    if (a.F <= 832) return launch_sweep_fb<832>(base, a, L, table_bytes, st);
    return launch_sweep_fb<1024>(base, a, L, table_bytes, st);
}

}  // namespace hdc
