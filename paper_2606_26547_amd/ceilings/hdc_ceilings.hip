// Ceiling probes of the device the hot path runs on, for reading the
// roofline fractions: the int8 matrix-core rate with random operands (the
// rate the chip sustains under that power draw, against the published
// dense peak) and the HBM read bandwidth of a plain streaming kernel
// (against the published 8 TB/s).  Measurement tools only: nothing on the
// hot path calls them.  Each entry point allocates, runs, times with HIP
// events and frees; it returns the rate, or a negative value on failure.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// CH independent accumulator chains per wave; the operands are random
// bytes loaded once (SH: the A operand's bytes reduced to 0 or 2, the
// shifted projection weights' statistics).  One MFMA = 32 x 32 x 32
// multiply-adds = 65536 ops.
template <int CH, int WPS, bool SH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPS))) void k_mfma(const v4i *src, int *out,
                                                                                          int iters)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    v4i a[4], b[4];
    for (int i = 0; i < 4; ++i) {
        a[i] = src[(t + 97 * i) & 65535];
        b[i] = src[(t * 7 + 31 * i) & 65535];
        if (SH)
            a[i] = (a[i] & 0x01010101) << 1;
    }
    v16i c[CH];
    for (int j = 0; j < CH; ++j)
        c[j] = v16i{};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int j = 0; j < CH; ++j)
                c[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[(s + j) & 3], b[s], c[j], 0, 0, 0);
    }
    int r = 0;
    for (int j = 0; j < CH; ++j)
        for (int v = 0; v < 16; ++v)
            r += c[j][v];
    out[t] = r;
}

// Read-only stream: 16 bytes per lane per step, grid-stride, one word
// written per thread at the end.
__global__ __launch_bounds__(256) void k_read(const uint4 *__restrict__ p, size_t n16, uint32_t *out)
{
    uint32_t acc = 0;
    const size_t step = (size_t)gridDim.x * 256;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * step < n16; i += 4 * step) {
        const uint4 a = p[i], b = p[i + step], c = p[i + 2 * step], d = p[i + 3 * step];
        acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n16; i += step) {
        const uint4 a = p[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

__global__ void k_fill(uint32_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        p[i] = (uint32_t)(i * 2654435761u) ^ 0x9e3779b9u;
}

template <class F>
double time_ms(F launch, int reps)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return -1.0;
    launch();
    if (hipDeviceSynchronize() != hipSuccess)
        return -1.0;
    (void)hipEventRecord(e0, 0);
    for (int r = 0; r < reps; ++r)
        launch();
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return hipGetLastError() == hipSuccess ? ms / reps : -1.0;
}

template <int CH, int WPS, bool SH>
double mfma_rate(int blocks_per_cu, int reps)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess)
        return -1.0;
    const int blocks = cus * blocks_per_cu;
    v4i *src = nullptr;
    int *out = nullptr;
    if (hipMalloc(&src, 65536 * sizeof(v4i)) != hipSuccess)
        return -1.0;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(int)) != hipSuccess) {
        (void)hipFree(src);
        return -1.0;
    }
    hipLaunchKernelGGL(k_fill, dim3(256), dim3(256), 0, 0, (uint32_t *)src, (size_t)65536 * 4);
    const int iters = 4096 / CH;
    const double ms = time_ms([&] { hipLaunchKernelGGL((k_mfma<CH, WPS, SH>), dim3(blocks), dim3(256), 0, 0, src,
                                                       out, iters); }, reps);
    (void)hipFree(src);
    (void)hipFree(out);
    if (ms <= 0)
        return -1.0;
    return (double)blocks * 4 * iters * 4 * CH * 65536.0 / (ms * 1e-3) / 1e12;
}

template <bool SH>
double mfma_i8(int chains, int waves_per_simd, int reps)
{
    const int b = waves_per_simd == 2 ? 2 : 1;
    if (waves_per_simd == 2) {
        switch (chains) {
        case 2: return mfma_rate<2, 2, SH>(b, reps);
        case 4: return mfma_rate<4, 2, SH>(b, reps);
        }
        return -1.0;
    }
    switch (chains) {
    case 1: return mfma_rate<1, 1, SH>(b, reps);
    case 2: return mfma_rate<2, 1, SH>(b, reps);
    case 4: return mfma_rate<4, 1, SH>(b, reps);
    case 8: return mfma_rate<8, 1, SH>(b, reps);
    }
    return -1.0;
}

}  // namespace

extern "C" {

// Sustained int8 matrix-core rate in TOP/s (1e12 integer ops per second) of
// a loop of v_mfma_i32_32x32x32_i8 on random operands: `chains` (1, 2, 4
// or 8) independent accumulators per wave, one or two waves per SIMD.
double hdc_ceiling_mfma_i8(int chains, int waves_per_simd, int reps)
{
    return mfma_i8<false>(chains, waves_per_simd, reps);
}

// The same loop with the A operand's bytes 0 or 2 (random), as the shifted
// projection weights are, the B operand random bytes as before.
double hdc_ceiling_mfma_i8_shifted(int chains, int waves_per_simd, int reps)
{
    return mfma_i8<true>(chains, waves_per_simd, reps);
}

// HBM read bandwidth in GB/s of a streaming kernel over `bytes` (rounded
// down to 16) of device memory, `blocks_per_cu` workgroups of 256 per CU.
double hdc_ceiling_hbm_read(size_t bytes, int blocks_per_cu, int reps)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess)
        return -1.0;
    const size_t n16 = bytes / 16;
    const int blocks = cus * (blocks_per_cu > 0 ? blocks_per_cu : 1);
    uint4 *p = nullptr;
    uint32_t *out = nullptr;
    if (hipMalloc(&p, n16 * 16) != hipSuccess)
        return -1.0;
    if (hipMalloc(&out, (size_t)blocks * 256 * 4) != hipSuccess) {
        (void)hipFree(p);
        return -1.0;
    }
    hipLaunchKernelGGL(k_fill, dim3(4096), dim3(256), 0, 0, (uint32_t *)p, n16 * 4);
    const double ms = time_ms([&] { hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, 0, p, n16, out); },
                              reps);
    (void)hipFree(p);
    (void)hipFree(out);
    if (ms <= 0)
        return -1.0;
    return (double)(n16 * 16) / (ms * 1e-3) / 1e9;
}

}  // extern "C"
