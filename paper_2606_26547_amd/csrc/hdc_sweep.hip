// hdc_eval_configs: one persistent launch that classifies the same queries
// under many approximation configurations (the inner loop of the tuning
// system: run each candidate, read back its accuracy and time).
//
// Workspace layout (all offsets 256-byte aligned):
//   [0]            queue counter (uint32)
//   [256]          the configurations as passed (copied from the host)
//   [..]           slot descriptors, ncfg x SlotDesc
//   [..]           slot order (longest first), ncfg x int32
//   [..]           first work item of each slot in that order, ncfg + 1 x int32
//   [..]           per-slot results as counted (correct, n, device ticks)
//   [..]           per-slot results as returned (correct, n, device_us)
//   [..]           per-slot class operand regions of fixed size
//                  (chunks(D) * KT KiB table + 128 int32 popcounts)
// Work item i belongs to the slot whose item range holds it (a binary search
// over the item offsets); a workgroup takes items from the queue until it is
// exhausted, so every workgroup reaches the exit whatever the grid size.
#include <string.h>

#include "hdc_encoder.h"

namespace hdc {

struct SlotDesc {
    int32_t s0, stride, nd, ct;   // ct < 0: invalid configuration (no work)
    int32_t iq;                   // work items: 1 = 128 queries, 2 = 256, 3 = 256 on the direct-staged body
    int32_t tiles;                // work items of the slot
    int64_t cost;
};

// Per-slot counters of the persistent kernel.
struct SlotCount {
    int32_t correct, n;
    uint64_t ticks;
};

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Class tiles compiled into the sweep kernel: 1 (K <= 32) or 4 (K <= 128).
// A slot's table holds whole pairs of 32-dimension chunks (the direct-staged
// 2x2 body reads them in pairs; the pad chunk is zero).
inline size_t sweep_table_bytes(int D, int K) { return (size_t)table_chunks(D) * sweep_kt(K) * 1024; }

struct SweepLayout {
    size_t off_cfg, off_desc, off_order, off_items, off_count, off_res, off_regions, region, total;
    SweepLayout(int ncfg, int D, int K)
    {
        off_cfg = 256;
        off_desc = align256(off_cfg + (size_t)ncfg * sizeof(hdc_config));
        off_order = align256(off_desc + (size_t)ncfg * sizeof(SlotDesc));
        off_items = align256(off_order + (size_t)ncfg * 4);
        off_count = align256(off_items + (size_t)(ncfg + 1) * 4);
        off_res = align256(off_count + (size_t)ncfg * sizeof(SlotCount));
        off_regions = align256(off_res + (size_t)ncfg * sizeof(hdc_config_result));
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

// Exclusive prefix sums over the block of one value per thread (at most 16
// waves); `wt` is LDS of 16 ints; returns the block total in *total.
__device__ __forceinline__ int block_exscan(int v, int *wt, int *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int s = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(s, o);
        if (lane >= o)
            s += u;
    }
    if (lane == 63)
        wt[wave] = s;
    __syncthreads();
    int base = 0, all = 0;
    for (int w = 0; w < nw; ++w) {
        base += w < wave ? wt[w] : 0;
        all += wt[w];
    }
    __syncthreads();
    *total = all;
    return base + s - v;
}

// Validate configurations, zero the counters, order the slots by decreasing
// cost (dimensions x compute cost; ties keep slot order) and lay out their
// work items in that order.  One block of 1024 threads.
__global__ __launch_bounds__(1024) void k_sweep_setup(int ncfg, int D, int64_t n, int x_type, int K,
                                                      uint8_t *__restrict__ ws, SweepLayout L)
{
    __shared__ int wt[16];
    const hdc_config *cfgs = (const hdc_config *)(ws + L.off_cfg);
    SlotDesc *desc = (SlotDesc *)(ws + L.off_desc);
    int32_t *order = (int32_t *)(ws + L.off_order);
    int32_t *items = (int32_t *)(ws + L.off_items);
    SlotCount *cnt = (SlotCount *)(ws + L.off_count);
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
        // built-in work items: 256 queries
        s.iq = c.tile_id == SV_ITEM128 ? 1 : c.tile_id == SV_ITEM256_DMA ? 3 : 2;
        s.tiles = ok ? (int32_t)((n + (s.iq == 1 ? 127 : 255)) / (s.iq == 1 ? 128 : 256)) : 0;
        desc[i] = s;
        cnt[i].correct = 0;
        cnt[i].n = ok ? (int32_t)n : 0;
        cnt[i].ticks = 0;
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
    __syncthreads();
    // first item of each rank: thread t covers ranks [t * per, (t + 1) * per)
    const int per = (ncfg + blockDim.x - 1) / blockDim.x;
    const int r0 = threadIdx.x * per;
    int local = 0;
    for (int r = r0; r < r0 + per && r < ncfg; ++r)
        local += desc[order[r]].tiles;
    int total;
    int run = block_exscan(local, wt, &total);
    for (int r = r0; r < r0 + per && r < ncfg; ++r) {
        items[r] = run;
        run += desc[order[r]].tiles;
    }
    if (threadIdx.x == 0)
        items[ncfg] = total;
}

// Per-slot results in the returned form: device time in microseconds.
__global__ __launch_bounds__(256) void k_sweep_results(int ncfg, const uint8_t *__restrict__ ws, SweepLayout L,
                                                       double us_per_tick)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ncfg)
        return;
    const SlotCount c = ((const SlotCount *)(ws + L.off_count))[i];
    hdc_config_result r;
    r.correct = c.correct;
    r.n = c.n;
    r.device_us = (double)c.ticks * us_per_tick;
    ((hdc_config_result *)(ws + L.off_res))[i] = r;
}

// Class operand tables of every slot (same layout as hdc_classify's).
__global__ __launch_bounds__(256) void k_sweep_tables(const uint64_t *__restrict__ C, int K, int64_t ldc,
                                                      uint8_t *__restrict__ ws, SweepLayout L, int KT,
                                                      int64_t per_slot)
{
    const int slot = blockIdx.y;
    const SlotDesc s = ((const SlotDesc *)(ws + L.off_desc))[slot];
    int8_t *tab = (int8_t *)(ws + L.off_regions + L.region * slot);
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
    const int slot = blockIdx.y, k = blockIdx.x;
    const SlotDesc s = ((const SlotDesc *)(ws + L.off_desc))[slot];
    int32_t *popc = (int32_t *)(ws + L.off_regions + L.region * slot + table_bytes);
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

// The fused classifier's direct-staged 2x2 body on one 256-query item
// (int8 features on the int8 path).
template <int KS, int KT>
__device__ __forceinline__ void sweep_pass_dma(EncodeArgs &a, uint8_t *smem, int64_t qblock, const int32_t *truth,
                                               SlotCount *res)
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
                                                     SlotCount *res)
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

// The persistent kernel.  Each slot runs with its own work-item size (its
// configuration's tile id); the LDS holds the largest body of the bucket.
template <int FB, int KT>
__global__ __launch_bounds__(256) void k_sweep(EncodeArgs base, const int32_t *__restrict__ truth,
                                               uint8_t *__restrict__ ws, SweepLayout L, size_t table_bytes,
                                               int ncfg)
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
        a.ctab = (const int8_t *)(ws + L.off_regions + L.region * slot);
        a.cpop = (const int32_t *)(ws + L.off_regions + L.region * slot + table_bytes);
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
            else
                sweep_item<C_FP8, FB / 64, KT, 2>(a, smem, qblock, truth, res);
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
                       a.ncfg);
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
    const SweepLayout L(a.ncfg, a.D, a.K);
    const int KT = sweep_kt(a.K);
    const size_t table_bytes = sweep_table_bytes(a.D, a.K);
    // the configurations go up with the other work of the stream (from
    // pageable memory the runtime stages them before returning)
    hipError_t e = hipMemcpyAsync(a.ws + L.off_cfg, a.cfgs, (size_t)a.ncfg * sizeof(hdc_config),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sweep_setup, dim3(1), dim3(1024), 0, st, a.ncfg, a.D, a.n, a.x_type, a.K, a.ws, L);
    const int64_t per_slot = table_chunks(a.D) * KT * 64;
    const unsigned gx = (unsigned)((per_slot + 255) / 256 < 1024 ? (per_slot + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_sweep_tables, dim3(gx, a.ncfg), dim3(256), 0, st, a.C, a.K, a.ldc, a.ws, L, KT, per_slot);
    hipLaunchKernelGGL(k_sweep_popc, dim3(KT * 32, a.ncfg), dim3(256), 0, st, a.C, a.K, a.ldc, a.ws, L,
                       table_bytes);
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
    if (a.F <= 128) e = launch_sweep_fb<128>(base, a, L, table_bytes, st);
    else if (a.F <= 256) e = launch_sweep_fb<256>(base, a, L, table_bytes, st);
    else if (a.F <= 512) e = launch_sweep_fb<512>(base, a, L, table_bytes, st);
    else if (a.F <= 640) e = launch_sweep_fb<640>(base, a, L, table_bytes, st);
    else if (a.F <= 832) e = launch_sweep_fb<832>(base, a, L, table_bytes, st);
    else e = launch_sweep_fb<1024>(base, a, L, table_bytes, st);
    if (e != hipSuccess)
        return e;
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
