// Retraining: integer class accumulators and one epoch of updates from the
// mispredicted training rows, then re-binarisation.  For every row i with
// pred[i] != labels[i], the row's bipolar hypervector b_i (+1 for bit 0,
// -1 for bit 1) is added to acc[labels[i]] and subtracted from
// acc[pred[i]]; without predictions (initialisation) every row adds b_i to
// its own class.  The model bit of (k, d) is 1 exactly when acc[k][d] < 0.
#include "hdc_device.h"

namespace hdc {

constexpr int kAccRows = 2048;   // rows per workgroup

// Grid over (word column w, block of kAccRows rows).  Each wave walks rows;
// lane j adds +-1 for bit j of the row's word into LDS counters of the
// affected classes; integer atomics keep the sums order-free.  Wrong rows
// are counted by the w == 0 workgroups.
__global__ __launch_bounds__(256) void k_acc_update(const uint64_t *__restrict__ H, int64_t n, int nbits,
                                                    int64_t ldh, const int32_t *__restrict__ labels,
                                                    const int32_t *__restrict__ pred, int K, int W,
                                                    int32_t *__restrict__ acc, int32_t *__restrict__ n_wrong)
{
    __shared__ int lacc[kMaxK * 64];
    __shared__ int lwrong;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int w = blockIdx.x % W;
    const int64_t r0 = (int64_t)(blockIdx.x / W) * kAccRows;
    for (int i = t; i < K * 64; i += 256)
        lacc[i] = 0;
    if (t == 0)
        lwrong = 0;
    __syncthreads();
    const int64_t r1 = r0 + kAccRows < n ? r0 + kAccRows : n;
    for (int64_t i = r0 + wave; i < r1; i += kWaves) {
        const int y = labels[i];
        const int p = pred ? pred[i] : -1;
        if (y < 0 || y >= K || (pred && (p == y || p < 0 || p >= K)))
            continue;
        const int b = 1 - 2 * (int)((H[i * ldh + w] >> lane) & 1ull);
        atomicAdd(&lacc[y * 64 + lane], b);
        if (pred) {
            atomicAdd(&lacc[p * 64 + lane], -b);
            if (w == 0 && lane == 0)
                atomicAdd(&lwrong, 1);
        }
    }
    __syncthreads();
    for (int i = t; i < K * 64; i += 256) {
        const int k = i >> 6, j = i & 63;
        const int d = w * 64 + j;
        if (d < nbits && lacc[i])
            atomicAdd(&acc[(int64_t)k * nbits + d], lacc[i]);
    }
    if (w == 0 && t == 0 && n_wrong && lwrong)
        atomicAdd(n_wrong, lwrong);
}

__global__ __launch_bounds__(256) void k_acc_binarize(const int32_t *__restrict__ acc, int K, int nbits, int W,
                                                      uint64_t *__restrict__ C, int64_t ldc)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)K * W)
        return;
    const int k = (int)(idx / W), w = (int)(idx % W);
    uint64_t word = 0;
    for (int j = 0; j < 64; ++j) {
        const int d = w * 64 + j;
        if (d < nbits && acc[(int64_t)k * nbits + d] < 0)
            word |= 1ull << j;
    }
    C[(int64_t)k * ldc + w] = word;
}

__global__ __launch_bounds__(256) void k_fill_zero_i32(int32_t *__restrict__ p, int64_t count)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx < count)
        p[idx] = 0;
}

hipError_t launch_retrain(const uint64_t *H, int64_t n, int nbits, int64_t ldh, const int32_t *labels,
                          const int32_t *pred, int K, int32_t *acc, uint64_t *C, int64_t ldc, int32_t *n_wrong,
                          hipStream_t st)
{
    const int W = (nbits + 63) / 64;
    if (!pred) {   // initialisation: acc = 0 first
        const int64_t cnt = (int64_t)K * nbits;
        hipLaunchKernelGGL(k_fill_zero_i32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, acc, cnt);
    }
    if (n_wrong)
        hipLaunchKernelGGL(k_fill_zero_i32, dim3(1), dim3(256), 0, st, n_wrong, (int64_t)1);
    const int64_t rb = (n + kAccRows - 1) / kAccRows;
    if (rb > 0)
        hipLaunchKernelGGL(k_acc_update, dim3((unsigned)(rb * W)), dim3(256), 0, st, H, n, nbits, ldh, labels, pred,
                           K, W, acc, n_wrong);
    hipLaunchKernelGGL(k_acc_binarize, dim3((unsigned)(((int64_t)K * W + 255) / 256)), dim3(256), 0, st, acc, K,
                       nbits, W, C, ldc);
    return hipGetLastError();
}

}  // namespace hdc
