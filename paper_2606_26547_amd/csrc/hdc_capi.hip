// C ABI of libhdc.so: argument validation and launch of the gfx950 kernels.
// Nothing here allocates device memory; every scratch byte comes from the
// caller's workspace.
#include <string.h>

#include "hdc_internal.h"

namespace hdc {
hipError_t launch_encode_i8(const EncodeArgs &a, int mode, Tile tile, hipStream_t st);
hipError_t launch_encode_fp8(const EncodeArgs &a, int mode, Tile tile, hipStream_t st);
hipError_t launch_encode_bf16(const EncodeArgs &a, int mode, Tile tile, hipStream_t st);
hipError_t launch_encode_f32(const EncodeArgs &a, int mode, Tile tile, hipStream_t st);
hipError_t launch_encode_fp8s(const EncodeArgs &a, int mode, Tile tile, hipStream_t st);

hipError_t launch_encode(const EncodeArgs &a, int compute, int mode, Tile tile, hipStream_t st)
{
    switch (compute) {
    case C_I8: return launch_encode_i8(a, mode, tile, st);
    case C_FP8: return launch_encode_fp8(a, mode, tile, st);
    case C_BF16: return launch_encode_bf16(a, mode, tile, st);
    case C_F32: return launch_encode_f32(a, mode, tile, st);
    case C_FP8S: return launch_encode_fp8s(a, mode, tile, st);
    case C_I8S: {
        EncodeArgs b = a;
        b.poff = 1;
        return launch_encode_i8(b, mode, tile, st);
    }
    case C_FP8H: {
        EncodeArgs b = a;
        b.poff = 1;
        return launch_encode_fp8(b, mode, tile, st);
    }
    }
    return hipErrorInvalidValue;
}
}  // namespace hdc

using namespace hdc;

namespace {

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Feature storage type of an hdc_dtype used as x_type, or -1.
int xtype_of(hdc_dtype t)
{
    switch (t) {
    case HDC_INT8: return X_INT8;
    case HDC_UINT8: return X_UINT8;
    case HDC_FP32: return X_FP32;
    default: return -1;
    }
}

// Kernel compute type for a (feature, compute) pair, or -1 if unsupported.
int compute_of(hdc_dtype x, hdc_dtype c)
{
    const bool integer = x == HDC_INT8 || x == HDC_UINT8;
    if (integer) {
        if (c == HDC_INT8) return C_I8;
        if (c == HDC_BF16) return C_BF16;
        if (c == HDC_FP8_E4M3) return C_FP8;
        if (c == HDC_FP8_E4M3_SPLIT) return C_FP8S;
        if (c == HDC_INT8_SHIFTED) return x == HDC_INT8 ? C_I8S : -1;
        if (c == HDC_FP8_E4M3_SHIFTED) return C_FP8H;
        return -1;
    }
    if (x == HDC_FP32) {
        if (c == HDC_FP32) return C_F32;
        if (c == HDC_BF16) return C_BF16;
        if (c == HDC_FP8_E4M3) return C_FP8;
    }
    return -1;
}

int32_t dims_count(hdc_dims d)
{
    if (d.stride < 1 || d.start < 0 || d.end <= d.start)
        return 0;
    return (int32_t)(((int64_t)d.end - d.start + d.stride - 1) / d.stride);
}

hdc_status from_hip(hipError_t e) { return e == hipSuccess ? HDC_OK : HDC_ERR_DEVICE; }

// Shared checks of the feature / projection operands.
hdc_status check_encode_operands(const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                                 const int8_t *P, int32_t D, int64_t ldp, hdc_dtype compute, hdc_dims dims,
                                 int *ct, int *xt)
{
    if (n < 0 || F <= 0 || D <= 0)
        return HDC_ERR_INVALID;
    *xt = xtype_of(x_type);
    *ct = compute_of(x_type, compute);
    if (*xt < 0)
        return HDC_ERR_INVALID;
    if (*ct < 0)
        return HDC_ERR_UNSUPPORTED;
    if (F > (*xt == X_FP32 ? kMaxFFloat : kMaxF))
        return HDC_ERR_UNSUPPORTED;
    if (dims.stride < 1 || dims.start < 0 || dims.end <= dims.start || dims.end > D)
        return HDC_ERR_INVALID;
    if (!P || ldp < round_up(F, 64) || ldp % 16 || !aligned(P, 16))
        return HDC_ERR_INVALID;
    // the encoders address P with 32-bit byte offsets (the direct-to-LDS
    // loads take a 32-bit voffset): every row must start below 2^32 - ldp
    if ((uint64_t)D * (uint64_t)ldp > (uint64_t)UINT32_MAX - (uint64_t)ldp)
        return HDC_ERR_UNSUPPORTED;
    if (n > 0 && (!X || ldx < round_up(F, 64) || ldx % 16 || !aligned(X, 16)))
        return HDC_ERR_INVALID;
    return HDC_OK;
}

EncodeArgs make_args(const void *X, int xt, int64_t n, int32_t F, int64_t ldx, const int8_t *P, int64_t ldp,
                     hdc_dims dims)
{
    EncodeArgs a;
    memset(&a, 0, sizeof a);
    a.X = X;
    a.x_type = xt;
    a.n = n;
    a.F = F;
    a.ldx = ldx;
    a.P = P;
    a.ldp = ldp;
    a.s0 = dims.start;
    a.stride = dims.stride;
    a.nd = dims_count(dims);
    return a;
}

}  // namespace

extern "C" {

const char *hdc_status_string(hdc_status s)
{
    switch (s) {
    case HDC_OK: return "HDC_OK";
    case HDC_ERR_INVALID: return "HDC_ERR_INVALID: invalid argument";
    case HDC_ERR_UNSUPPORTED: return "HDC_ERR_UNSUPPORTED: type pair or size not supported";
    case HDC_ERR_WORKSPACE: return "HDC_ERR_WORKSPACE: workspace too small or misaligned";
    case HDC_ERR_DEVICE: return "HDC_ERR_DEVICE: kernel launch failed";
    }
    return "unknown hdc_status";
}

int32_t hdc_dims_count(hdc_dims dims) { return dims_count(dims); }

hdc_status hdc_encode_tiled(void *stream, const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                            const int8_t *P, int32_t D, int64_t ldp, hdc_dtype compute, hdc_dims dims, uint64_t *H,
                            int64_t ldh, int32_t tile)
{
    int ct, xt;
    hdc_status s = check_encode_operands(X, x_type, n, F, ldx, P, D, ldp, compute, dims, &ct, &xt);
    if (s != HDC_OK)
        return s;
    const int32_t nd = dims_count(dims);
    if (n > 0 && (!H || ldh < (nd + 63) / 64 || !aligned(H, 8)))
        return HDC_ERR_INVALID;
    if (tile < 0 || !tile_compiled(KK_ENCODE, xt, ct, F, 1, tile))
        return HDC_ERR_UNSUPPORTED;
    if (n == 0)
        return HDC_OK;
    EncodeArgs a = make_args(X, xt, n, F, ldx, P, ldp, dims);
    a.H32 = (uint32_t *)H;
    a.ldh32 = 2 * ldh;
    a.max_split = 1 << 30;   // the splits write disjoint words: no scratch
    return from_hip(launch_encode(a, ct, M_ENCODE, Tile{tile}, (hipStream_t)stream));
}

hdc_status hdc_encode(void *stream, const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                      const int8_t *P, int32_t D, int64_t ldp, hdc_dtype compute, hdc_dims dims, uint64_t *H,
                      int64_t ldh)
{
    return hdc_encode_tiled(stream, X, x_type, n, F, ldx, P, D, ldp, compute, dims, H, ldh, 0);
}

hdc_status hdc_shift_projection(void *stream, const int8_t *P, int32_t D, int32_t F, int64_t ldp, hdc_dtype compute,
                                int8_t *out, int64_t ldo)
{
    if (D <= 0 || F <= 0)
        return HDC_ERR_INVALID;
    if (compute != HDC_INT8_SHIFTED && compute != HDC_FP8_E4M3_SHIFTED)
        return HDC_ERR_UNSUPPORTED;
    if (F > kMaxF)
        return HDC_ERR_UNSUPPORTED;
    if (!P || ldp < round_up(F, 64) || ldp % 16 || !aligned(P, 16))
        return HDC_ERR_INVALID;
    if (!out || ldo < round_up(F, 64) || ldo % 16 || !aligned(out, 16))
        return HDC_ERR_INVALID;
    if ((uint64_t)D * (uint64_t)ldo > (uint64_t)UINT32_MAX - (uint64_t)ldo)
        return HDC_ERR_UNSUPPORTED;
    // in place only with the same pitch: each unit is read and written by one thread
    const uintptr_t p0 = (uintptr_t)P, p1 = p0 + (uintptr_t)((int64_t)D * ldp);
    const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (uintptr_t)((int64_t)D * ldo);
    if (o0 < p1 && p0 < o1 && !(o0 == p0 && ldo == ldp))
        return HDC_ERR_INVALID;
    return from_hip(launch_shift_projection(P, D, F, ldp, compute == HDC_FP8_E4M3_SHIFTED, out, ldo,
                                            (hipStream_t)stream));
}

size_t hdc_bundle_workspace_bytes(int64_t n, int32_t nbits, int32_t K)
{
    if (n < 0 || nbits <= 0 || K <= 0 || K > kMaxK || !group_count_fits(n))
        return 0;
    return group_count_ws_bytes(0, n, nbits, K);
}

static hdc_status check_bundle(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh, const int32_t *labels,
                               int32_t K, const uint64_t *C, int64_t ldc)
{
    if (n < 0 || nbits <= 0 || K <= 0)
        return HDC_ERR_INVALID;
    if (K > kMaxK || !group_count_fits(n))
        return HDC_ERR_UNSUPPORTED;
    const int64_t W = (nbits + 63) / 64;
    if (!C || ldc < W || (n > 0 && (!H || !labels || ldh < W || !aligned(H, 8))))
        return HDC_ERR_INVALID;
    return HDC_OK;
}

hdc_status hdc_bundle(void *stream, const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                      const int32_t *labels, int32_t K, uint64_t *C, int64_t ldc, int32_t *counts, void *ws,
                      size_t ws_bytes)
{
    const hdc_status s = check_bundle(H, n, nbits, ldh, labels, K, C, ldc);
    if (s != HDC_OK)
        return s;
    if (!ws || ws_bytes < hdc_bundle_workspace_bytes(n, nbits, K) || !aligned(ws, 256))
        return HDC_ERR_WORKSPACE;
    return from_hip(launch_group_count(0, H, n, nbits, ldh, labels, nullptr, K, nullptr, C, ldc, counts, nullptr, ws,
                                       (hipStream_t)stream));
}

size_t hdc_bundle_noalloc_limit_bytes(void) { return kNoAllocScratchBytes; }

hdc_status hdc_bundle_noalloc(void *stream, const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                              const int32_t *labels, int32_t K, uint64_t *C, int64_t ldc, int32_t *counts)
{
    const hdc_status s = check_bundle(H, n, nbits, ldh, labels, K, C, ldc);
    if (s != HDC_OK)
        return s;
    if (hdc_bundle_workspace_bytes(n, nbits, K) > kNoAllocScratchBytes)
        return HDC_ERR_UNSUPPORTED;
    void *ws = nullptr;
    const hipError_t e = noalloc_scratch(&ws);
    if (e != hipSuccess)
        return HDC_ERR_DEVICE;
    return from_hip(launch_group_count(0, H, n, nbits, ldh, labels, nullptr, K, nullptr, C, ldc, counts, nullptr, ws,
                                       (hipStream_t)stream));
}

hdc_status hdc_hamming_argmin(void *stream, const uint64_t *Q, int64_t n, int64_t ldq, const uint64_t *C,
                              int32_t K, int64_t ldc, int32_t nbits, hdc_dims perf, int32_t *argmin,
                              int32_t *min_dist, int32_t *dists)
{
    if (n < 0 || K <= 0 || nbits <= 0)
        return HDC_ERR_INVALID;
    if (perf.stride < 1 || perf.start < 0 || perf.end <= perf.start || perf.end > nbits)
        return HDC_ERR_INVALID;
    if (K > kMaxK || perf.end > 65536)
        return HDC_ERR_UNSUPPORTED;
    const int64_t W = ((int64_t)nbits + 63) / 64;
    if (!C || ldc < W)
        return HDC_ERR_INVALID;
    if (n == 0)
        return HDC_OK;
    if (!Q || ldq < W || !argmin)
        return HDC_ERR_INVALID;
    return from_hip(launch_hamming(Q, n, ldq, C, K, ldc, perf.start, perf.end, perf.stride, argmin, min_dist,
                                   dists, (hipStream_t)stream));
}

static hdc_status check_retrain(const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh, const int32_t *labels,
                                int32_t K, const int32_t *acc, const uint64_t *C, int64_t ldc, const void *ws,
                                size_t ws_bytes)
{
    if (n < 0 || nbits <= 0 || K <= 0)
        return HDC_ERR_INVALID;
    if (K > kMaxK || !group_count_fits(n))
        return HDC_ERR_UNSUPPORTED;
    const int64_t W = (nbits + 63) / 64;
    if (!acc || !aligned(acc, 4) || !C || ldc < W || (n > 0 && (!H || !labels || ldh < W || !aligned(H, 8))))
        return HDC_ERR_INVALID;
    if (!ws || ws_bytes < hdc_retrain_workspace_bytes(n, nbits, K) || !aligned(ws, 256))
        return HDC_ERR_WORKSPACE;
    return HDC_OK;
}

size_t hdc_retrain_workspace_bytes(int64_t n, int32_t nbits, int32_t K)
{
    if (n < 0 || nbits <= 0 || K <= 0 || K > kMaxK || !group_count_fits(n))
        return 0;
    const size_t a = group_count_ws_bytes(1, n, nbits, K), b = group_count_ws_bytes(2, n, nbits, K);
    return a > b ? a : b;
}

hdc_status hdc_class_acc(void *stream, const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                         const int32_t *labels, int32_t K, int32_t *acc, uint64_t *C, int64_t ldc, void *ws,
                         size_t ws_bytes)
{
    const hdc_status s = check_retrain(H, n, nbits, ldh, labels, K, acc, C, ldc, ws, ws_bytes);
    if (s != HDC_OK)
        return s;
    return from_hip(launch_group_count(1, H, n, nbits, ldh, labels, nullptr, K, acc, C, ldc, nullptr, nullptr, ws,
                                       (hipStream_t)stream));
}

hdc_status hdc_retrain_epoch(void *stream, const uint64_t *H, int64_t n, int32_t nbits, int64_t ldh,
                             const int32_t *labels, const int32_t *pred, int32_t K, int32_t *acc, uint64_t *C,
                             int64_t ldc, int32_t *n_wrong, void *ws, size_t ws_bytes)
{
    const hdc_status s = check_retrain(H, n, nbits, ldh, labels, K, acc, C, ldc, ws, ws_bytes);
    if (s != HDC_OK)
        return s;
    if (n > 0 && !pred)
        return HDC_ERR_INVALID;
    return from_hip(launch_group_count(2, H, n, nbits, ldh, labels, pred, K, acc, C, ldc, nullptr, n_wrong, ws,
                                       (hipStream_t)stream));
}

hdc_status hdc_adc_argmax(void *stream, const uint64_t *Q, int64_t n, int64_t ldq, const uint64_t *C, int32_t K,
                          int64_t ldc, hdc_dims perf, hdc_adc adc, int32_t *label, int32_t *max_score,
                          int32_t *scores)
{
    if (n < 0 || K <= 0)
        return HDC_ERR_INVALID;
    if (K > kMaxK || perf.end > 65536)
        return HDC_ERR_UNSUPPORTED;
    if (perf.stride < 1 || perf.start < 0 || perf.end <= perf.start)
        return HDC_ERR_INVALID;
    if (adc.res_bits < 1 || adc.res_bits > 16 || adc.step < 1 || adc.floor > adc.ceil)
        return HDC_ERR_INVALID;
    const int64_t W = (perf.end + 63) / 64;
    if (!C || ldc < W)
        return HDC_ERR_INVALID;
    if (n == 0)
        return HDC_OK;
    if (!Q || ldq < W || !label)
        return HDC_ERR_INVALID;
    return from_hip(launch_adc_argmax(Q, n, ldq, C, K, ldc, perf.start, perf.end, perf.stride, adc.res_bits,
                                      adc.step, adc.floor, adc.ceil, label, max_score, scores,
                                      (hipStream_t)stream));
}

static hdc_status check_perf(hdc_dims perf, int32_t K)
{
    if (K <= 0 || perf.stride < 1 || perf.start < 0 || perf.end <= perf.start)
        return HDC_ERR_INVALID;
    if (K > kMaxK || perf.end > 65536)
        return HDC_ERR_UNSUPPORTED;
    return HDC_OK;
}

size_t hdc_hamming_workspace_bytes(hdc_dims perf, int32_t K)
{
    if (check_perf(perf, K) != HDC_OK)
        return 0;
    return ham_workspace_bytes(perf.start, perf.end, K);
}

hdc_status hdc_hamming_prepare(void *stream, const uint64_t *C, int32_t K, int64_t ldc, hdc_dims perf, void *ws,
                               size_t ws_bytes)
{
    const hdc_status s = check_perf(perf, K);
    if (s != HDC_OK)
        return s;
    if (!C || ldc < (perf.end + 63) / 64)
        return HDC_ERR_INVALID;
    if (!ws || ws_bytes < hdc_hamming_workspace_bytes(perf, K) || !aligned(ws, 16))
        return HDC_ERR_WORKSPACE;
    return from_hip(launch_ham_prepare(C, K, ldc, perf.start, perf.end, perf.stride, (uint8_t *)ws,
                                       (hipStream_t)stream));
}

hdc_status hdc_hamming_argmin_prepared(void *stream, const uint64_t *Q, int64_t n, int64_t ldq, int32_t K,
                                       hdc_dims perf, int32_t *argmin, int32_t *min_dist, int32_t *dists,
                                       const void *ws, size_t ws_bytes)
{
    if (n < 0)
        return HDC_ERR_INVALID;
    const hdc_status s = check_perf(perf, K);
    if (s != HDC_OK)
        return s;
    if (!ws || ws_bytes < hdc_hamming_workspace_bytes(perf, K) || !aligned(ws, 16))
        return HDC_ERR_WORKSPACE;
    if (n == 0)
        return HDC_OK;
    if (!Q || ldq < (perf.end + 63) / 64 || ldq % 2 || !aligned(Q, 16) || !argmin)
        return HDC_ERR_INVALID;
    if (ldq > kMaxPreparedLdq)
        return HDC_ERR_UNSUPPORTED;
    return from_hip(launch_ham_prepared(Q, n, ldq, K, perf.start, perf.end, (const uint8_t *)ws, argmin,
                                        min_dist, dists, (hipStream_t)stream));
}

size_t hdc_cosine_workspace_bytes(hdc_dims perf, int32_t K)
{
    if (check_perf(perf, K) != HDC_OK)
        return 0;
    return cos_workspace_bytes(perf.start, perf.end, K);
}

hdc_status hdc_cosine_prepare(void *stream, const int32_t *acc, int32_t K, int64_t lda, hdc_dims perf, void *ws,
                              size_t ws_bytes)
{
    const hdc_status s = check_perf(perf, K);
    if (s != HDC_OK)
        return s;
    if (!acc || lda < perf.end)
        return HDC_ERR_INVALID;
    if (!ws || ws_bytes < hdc_cosine_workspace_bytes(perf, K) || !aligned(ws, 16))
        return HDC_ERR_WORKSPACE;
    return from_hip(launch_cos_prepare(acc, K, lda, perf.start, perf.end, perf.stride, (uint8_t *)ws,
                                       (hipStream_t)stream));
}

hdc_status hdc_cosine_argmax_prepared(void *stream, const uint64_t *Q, int64_t n, int64_t ldq, int32_t K,
                                      hdc_dims perf, int32_t *label, double *max_score, double *scores,
                                      const void *ws, size_t ws_bytes)
{
    if (n < 0)
        return HDC_ERR_INVALID;
    const hdc_status s = check_perf(perf, K);
    if (s != HDC_OK)
        return s;
    if (!ws || ws_bytes < hdc_cosine_workspace_bytes(perf, K) || !aligned(ws, 16))
        return HDC_ERR_WORKSPACE;
    if (n == 0)
        return HDC_OK;
    if (!Q || ldq < (perf.end + 63) / 64 || ldq % 2 || !aligned(Q, 16) || !label)
        return HDC_ERR_INVALID;
    if (ldq > kMaxPreparedLdq)
        return HDC_ERR_UNSUPPORTED;
    return from_hip(launch_cos_prepared(Q, n, ldq, K, perf.start, perf.end, (const uint8_t *)ws, label, max_score,
                                        scores, (hipStream_t)stream));
}

hdc_status hdc_feature_perforate(void *stream, const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                                 hdc_dims fperf, void *Y, int64_t ldy)
{
    if (n < 0 || F <= 0 || fperf.stride < 1 || fperf.start < 0 || fperf.end <= fperf.start || fperf.end > F)
        return HDC_ERR_INVALID;
    int elem;
    if (x_type == HDC_INT8 || x_type == HDC_UINT8)
        elem = 1;
    else if (x_type == HDC_FP32)
        elem = 4;
    else
        return HDC_ERR_UNSUPPORTED;
    const int32_t nf = dims_count(fperf);
    if (n == 0)
        return HDC_OK;
    if (!X || !Y || ldx < F || ldy < nf || (ldy * elem) % 16 || !aligned(Y, 16))
        return HDC_ERR_INVALID;
    return from_hip(launch_gather_cols(X, elem, n, ldx, fperf.start, fperf.stride, nf, Y, ldy, (hipStream_t)stream));
}

hdc_status hdc_level_quantize(void *stream, const float *X, int64_t n, int32_t F, int64_t ldx, const float *lo,
                              const float *hi, int32_t L, uint16_t *lev, int64_t ldl)
{
    if (n < 0 || F <= 0 || L < 1 || L > 65535)
        return HDC_ERR_INVALID;
    if (n == 0)
        return HDC_OK;
    if (!X || !lo || !hi || !lev || ldx < F || ldl < F)
        return HDC_ERR_INVALID;
    return from_hip(launch_level_quantize(X, n, F, ldx, lo, hi, L, lev, ldl, (hipStream_t)stream));
}

hdc_status hdc_level_id_encode(void *stream, const uint16_t *lev, int64_t n, int32_t F, int64_t ldl,
                               const uint64_t *ID, int64_t ldid, const uint64_t *LV, int32_t L, int64_t ldlv,
                               int32_t D, uint64_t *H, int64_t ldh)
{
    if (n < 0 || F <= 0 || L < 1 || D <= 0)
        return HDC_ERR_INVALID;
    if (F > kMaxLevelIdF || L > kMaxLevels)
        return HDC_ERR_UNSUPPORTED;
    const int64_t W = (D + 63) / 64;
    if (!ID || !LV || ldid < W || ldlv < W)
        return HDC_ERR_INVALID;
    if (n == 0)
        return HDC_OK;
    if (!lev || !H || ldl < (F + 7) / 8 * 8 || ldl % 8 || !aligned(lev, 16) || ldh < W)
        return HDC_ERR_INVALID;
    return from_hip(launch_level_id(lev, n, F, ldl, ID, ldid, LV, L, ldlv, D, H, ldh, (hipStream_t)stream));
}

// (kernel-side feature kind, compute type) of a tile-table bucket, false if
// the pair has no kernels
static bool tile_key(hdc_kernel kind, hdc_dtype x_type, hdc_dtype compute, int *xt, int *ct)
{
    *xt = xtype_of(x_type);
    if (*xt < 0)
        return false;
    if (kind == HDC_KERNEL_SWEEP) {
        *ct = C_I8;
        return *xt != X_FP32;
    }
    if (kind != HDC_KERNEL_ENCODE && kind != HDC_KERNEL_CLASSIFY)
        return false;
    *ct = compute_of(x_type, compute);
    return *ct >= 0;
}

int32_t hdc_tile_variants(hdc_kernel kind, hdc_dtype x_type, hdc_dtype compute, int32_t F, int32_t K,
                          int32_t *variants, int32_t cap)
{
    int xt, ct;
    if (!tile_key(kind, x_type, compute, &xt, &ct) || F <= 0 || (cap > 0 && !variants))
        return -1;
    int v[8];
    const int n = tile_variants((int)kind, xt, ct, F, kind == HDC_KERNEL_ENCODE ? 1 : K, v, 8);
    for (int i = 0; i < n && i < cap; ++i)
        variants[i] = v[i];
    return n;
}

size_t hdc_adc_workspace_bytes(hdc_dims perf, int32_t K)
{
    if (check_perf(perf, K) != HDC_OK)
        return 0;
    return adc_workspace_bytes(perf.start, perf.end, K);
}

hdc_status hdc_adc_prepare(void *stream, const uint64_t *C, int32_t K, int64_t ldc, hdc_dims perf, void *ws,
                           size_t ws_bytes)
{
    const hdc_status s = check_perf(perf, K);
    if (s != HDC_OK)
        return s;
    if (!C || ldc < (perf.end + 63) / 64)
        return HDC_ERR_INVALID;
    if (!ws || ws_bytes < hdc_adc_workspace_bytes(perf, K) || !aligned(ws, 16))
        return HDC_ERR_WORKSPACE;
    return from_hip(launch_adc_prepare(C, K, ldc, perf.start, perf.end, perf.stride, (uint8_t *)ws,
                                       (hipStream_t)stream));
}

hdc_status hdc_adc_argmax_prepared(void *stream, const uint64_t *Q, int64_t n, int64_t ldq, int32_t K,
                                   hdc_dims perf, hdc_adc adc, int32_t *label, int32_t *max_score, int32_t *scores,
                                   const void *ws, size_t ws_bytes)
{
    if (n < 0)
        return HDC_ERR_INVALID;
    const hdc_status s = check_perf(perf, K);
    if (s != HDC_OK)
        return s;
    if (adc.res_bits < 1 || adc.res_bits > 16 || adc.step < 1 || adc.floor > adc.ceil)
        return HDC_ERR_INVALID;
    if (!ws || ws_bytes < hdc_adc_workspace_bytes(perf, K) || !aligned(ws, 16))
        return HDC_ERR_WORKSPACE;
    if (n == 0)
        return HDC_OK;
    if (!Q || ldq < (perf.end + 63) / 64 || ldq % 2 || !aligned(Q, 16) || !label)
        return HDC_ERR_INVALID;
    if (ldq > kMaxPreparedLdq)
        return HDC_ERR_UNSUPPORTED;
    return from_hip(launch_adc_prepared(Q, n, ldq, K, perf.start, perf.end, adc.res_bits, adc.step, adc.floor,
                                        adc.ceil, (const uint8_t *)ws, label, max_score, scores,
                                        (hipStream_t)stream));
}

size_t hdc_classify_workspace_bytes(int32_t n_dims, int32_t K)
{
    if (n_dims <= 0 || K <= 0 || K > kMaxK)
        return 0;
    return class_table_bytes(n_dims, K) + 4 * 32 * 4;
}

hdc_status hdc_classify_prepare(void *stream, const uint64_t *C, int32_t K, int64_t ldc, hdc_dims dims, void *ws,
                                size_t ws_bytes)
{
    if (K <= 0 || dims.stride < 1 || dims.start < 0 || dims.end <= dims.start)
        return HDC_ERR_INVALID;
    if (K > kMaxK)
        return HDC_ERR_UNSUPPORTED;
    if (!C || ldc < (dims.end + 63) / 64)
        return HDC_ERR_INVALID;
    const int32_t nd = dims_count(dims);
    if (!ws || ws_bytes < hdc_classify_workspace_bytes(nd, K) || !aligned(ws, 16))
        return HDC_ERR_WORKSPACE;
    int8_t *tab = (int8_t *)ws;
    int32_t *cpop = (int32_t *)((uint8_t *)ws + class_table_bytes(nd, K));
    return from_hip(launch_class_table(C, K, ldc, dims.start, dims.stride, nd, tab, cpop, (hipStream_t)stream));
}

size_t hdc_classify_scratch_bytes(int64_t n, int32_t n_dims, int32_t K)
{
    if (n <= 0 || n_dims <= 0 || K <= 0 || K > kMaxK)
        return 0;
    // the most splits any variant takes (the largest query blocks, two
    // resident workgroups per CU)
    const int Z = split_count((n + kQpbMax - 1) / kQpbMax, n_dims, 1 << 30, kSplitTargetMax);
    return Z > 1 ? (size_t)4 * Z * K * n : 0;
}

hdc_status hdc_classify_prepared(void *stream, const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                                 const int8_t *P, int32_t D, int64_t ldp, hdc_dtype compute, hdc_dims dims,
                                 int32_t K, int32_t *labels, int32_t *dists, const void *ws, size_t ws_bytes,
                                 void *scratch, size_t scratch_bytes, int32_t tile)
{
    int ct, xt;
    hdc_status s = check_encode_operands(X, x_type, n, F, ldx, P, D, ldp, compute, dims, &ct, &xt);
    if (s != HDC_OK)
        return s;
    if (K <= 0)
        return HDC_ERR_INVALID;
    if (K > kMaxK)
        return HDC_ERR_UNSUPPORTED;
    if (n > 0 && !labels)
        return HDC_ERR_INVALID;
    const int32_t nd = dims_count(dims);
    if (!ws || ws_bytes < hdc_classify_workspace_bytes(nd, K) || !aligned(ws, 16))
        return HDC_ERR_WORKSPACE;
    if (scratch && !aligned(scratch, 4))
        return HDC_ERR_WORKSPACE;
    if (tile < 0 || !tile_compiled(KK_CLASSIFY, xt, ct, F, K, tile))
        return HDC_ERR_UNSUPPORTED;
    if (n == 0)
        return HDC_OK;
    EncodeArgs a = make_args(X, xt, n, F, ldx, P, ldp, dims);
    a.ctab = (const int8_t *)ws;
    a.cpop = (const int32_t *)((const uint8_t *)ws + class_table_bytes(nd, K));
    a.K = K;
    a.labels = labels;
    a.dists = dists;
    // dimension splits: as many as the scratch holds partial class sums for
    if (scratch) {
        const int64_t cap = (int64_t)(scratch_bytes / ((size_t)4 * K * n));
        a.max_split = (int32_t)(cap < (1 << 30) ? cap : (1 << 30));
        a.part = (int32_t *)scratch;
    }
    return from_hip(launch_encode(a, ct, M_CLASSIFY, Tile{tile}, (hipStream_t)stream));
}

hdc_status hdc_classify(void *stream, const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                        const int8_t *P, int32_t D, int64_t ldp, hdc_dtype compute, hdc_dims dims,
                        const uint64_t *C, int32_t K, int64_t ldc, int32_t *labels, int32_t *dists, void *ws,
                        size_t ws_bytes, void *scratch, size_t scratch_bytes, int32_t tile)
{
    int ct, xt;
    hdc_status s = check_encode_operands(X, x_type, n, F, ldx, P, D, ldp, compute, dims, &ct, &xt);
    if (s != HDC_OK)
        return s;
    if (K <= 0)
        return HDC_ERR_INVALID;
    if (n > 0 && !labels)
        return HDC_ERR_INVALID;
    if (n == 0) {
        const int32_t nd = dims_count(dims);
        if (K > kMaxK || tile < 0 || !tile_compiled(KK_CLASSIFY, xt, ct, F, K, tile))
            return HDC_ERR_UNSUPPORTED;
        if (!ws || ws_bytes < hdc_classify_workspace_bytes(nd, K))
            return HDC_ERR_WORKSPACE;
        return HDC_OK;
    }
    s = hdc_classify_prepare(stream, C, K, ldc, dims, ws, ws_bytes);
    if (s != HDC_OK)
        return s;
    return hdc_classify_prepared(stream, X, x_type, n, F, ldx, P, D, ldp, compute, dims, K, labels, dists, ws,
                                 ws_bytes, scratch, scratch_bytes, tile);
}

size_t hdc_eval_configs_workspace_bytes(int32_t ncfg, int32_t F, int32_t D, int32_t K)
{
    if (ncfg > kMaxConfigs)
        return 0;
    return sweep_workspace_bytes(ncfg, F, D, K);
}

hdc_status hdc_eval_configs(void *stream, const void *X, hdc_dtype x_type, int64_t n, int32_t F, int64_t ldx,
                            const int32_t *truth, const int8_t *P, int32_t D, int64_t ldp, const uint64_t *C,
                            int32_t K, int64_t ldc, const hdc_config *cfgs, int32_t ncfg,
                            hdc_config_result *out, void *ws, size_t ws_bytes, int32_t max_workgroups)
{
    int ct, xt;
    hdc_status s = check_encode_operands(X, x_type, n, F, ldx, P, D, ldp, HDC_INT8, hdc_dims{0, D, 1}, &ct, &xt);
    if (s != HDC_OK)
        return s;
    if (K <= 0 || ncfg <= 0 || max_workgroups < 0)
        return HDC_ERR_INVALID;
    if (K > kMaxK || ncfg > kMaxConfigs || xt == X_FP32)
        return HDC_ERR_UNSUPPORTED;
    if (!C || ldc < (D + 63) / 64 || !cfgs || !out || (n > 0 && !truth))
        return HDC_ERR_INVALID;
    for (int32_t i = 0; i < ncfg; ++i)
        if (cfgs[i].tile_id < 0 || !tile_compiled(KK_SWEEP, xt, C_I8, F, K, cfgs[i].tile_id))
            return HDC_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < hdc_eval_configs_workspace_bytes(ncfg, F, D, K) || !aligned(ws, 256))
        return HDC_ERR_WORKSPACE;
    if (n == 0) {
        for (int32_t i = 0; i < ncfg; ++i)
            out[i] = hdc_config_result{0, 0, 0.0};
        return HDC_OK;
    }
    SweepArgs a;
    a.X = X;
    a.x_type = xt;
    a.n = n;
    a.F = F;
    a.ldx = ldx;
    a.truth = truth;
    a.P = P;
    a.ldp = ldp;
    a.D = D;
    a.C = C;
    a.K = K;
    a.ldc = ldc;
    a.cfgs = cfgs;
    a.ncfg = ncfg;
    a.out = out;
    a.ws = (uint8_t *)ws;
    a.ws_bytes = ws_bytes;
    a.max_wg = max_workgroups;
    return from_hip(launch_sweep(a, (hipStream_t)stream));
}

double hdc_device_clock_hz(void)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0.0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return 0.0;
    return (double)khz * 1000.0;
}

hdc_status hdc_convert_features(void *stream, const void *X, hdc_dtype x_type, int64_t n, int32_t F,
                                int64_t ldx, hdc_dtype compute, float *out)
{
    const int xt = xtype_of(x_type), ct = compute_of(x_type, compute);
    if (n < 0 || F <= 0 || xt < 0)
        return HDC_ERR_INVALID;
    if (ct < 0)
        return HDC_ERR_UNSUPPORTED;
    if (n == 0)
        return HDC_OK;
    if (!X || !out || ldx < F)
        return HDC_ERR_INVALID;
    return from_hip(launch_convert(X, xt, n, F, ldx, ct, out, (hipStream_t)stream));
}

}  // extern "C"
