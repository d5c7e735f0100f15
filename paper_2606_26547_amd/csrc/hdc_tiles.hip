// Tile variants: which kernel shapes each (kernel, feature type, compute
// type, feature width, class tiles) bucket is compiled with.  A launch names
// its variant (0 = the built-in rule); an autotuner measures the variants of
// a bucket and passes the fastest with each call.  Every variant of a bucket
// computes the same result.  Nothing here is mutable.
#include "hdc_internal.h"

namespace hdc {

namespace {

constexpr int kNI = sizeof(kIntWidths) / sizeof(kIntWidths[0]);
constexpr int kNF = sizeof(kF32Widths) / sizeof(kF32Widths[0]);
constexpr int kNS = sizeof(kSweepWidths) / sizeof(kSweepWidths[0]);

// Variants a bucket is compiled with; the first listed is what 0 selects.
int encoder_variants(int ct, int x_type, int width, int kt, bool classify, int *out)
{
    const int ks = width / kstep_of(ct);
    int n = 0;
    if (ct == C_FP8H) {   // E4M3 on the shifted projection: the direct 2x2 shape
        if (x_type == X_FP32 || !shift8_tile(ks, kt))
            return 0;
        out[n++] = TV_DMA_2X2;
        return n;
    }
    if (ct == C_I8S) {   // the shifted projection: the shift_tile shapes only
        if (x_type != X_INT8 || !shift_tile(ks, kt))
            return 0;
        out[n++] = TV_DMA_2X2;
        if (classify && big3_tile(ks, kt))
            out[n++] = TV_DMA_2X3;
        return n;
    }
    if (ct == C_I8 && x_type == X_INT8) {
        if (big_tile(ks, kt))
            out[n++] = TV_DMA_2X2;
        out[n++] = TV_DMA_1X1;
        if (classify && big3_tile(ks, kt))
            out[n++] = TV_DMA_2X3;
    }
    if (qt2_fits(ct, ks))
        out[n++] = TV_REG_QT2;
    out[n++] = TV_REG_QT1;
    // the classifier compiles four class tiles with one query tile only
    if (kt == 4) {
        int m = 0;
        for (int i = 0; i < n; ++i)
            if (out[i] != TV_REG_QT2 && out[i] != TV_DMA_2X2)
                out[m++] = out[i];
        n = m;
    }
    return n;
}

bool encoder_bucket(int kind, int x_type, int ct, int F, int K)
{
    if ((kind != KK_ENCODE && kind != KK_CLASSIFY) || ct < 0 || ct >= kComputeTypes)
        return false;
    return width_index(x_type, F) >= 0 && K >= 1 && K <= kMaxK;
}

bool sweep_bucket(int F, int K) { return sweep_width_index(F) >= 0 && K >= 1 && K <= kMaxK; }

}  // namespace

int width_index(int x_type, int F)
{
    if (x_type == X_FP32) {
        for (int i = 0; i < kNF; ++i)
            if (F <= kF32Widths[i])
                return i;
        return -1;
    }
    for (int i = 0; i < kNI; ++i)
        if (F <= kIntWidths[i])
            return i;
    return -1;
}

int sweep_width_index(int F)
{
    for (int i = 0; i < kNS; ++i)
        if (F <= kSweepWidths[i])
            return i;
    return -1;
}

int tile_variants(int kind, int x_type, int ct, int F, int K, int *out, int cap)
{
    int v[8], n = 0;
    if (kind == KK_SWEEP) {
        if (!sweep_bucket(F, K) || x_type == X_FP32)
            return -1;
        v[n++] = SV_ITEM256;
        v[n++] = SV_ITEM128;
        const int wi = sweep_width_index(F);
        // the direct-staged bodies: up to 640 features, one class tile (int8
        // configurations take them with int8 features only)
        if (sweep_kt(K) == 1 && kSweepWidths[wi] <= 640)
            v[n++] = SV_ITEM256_DMA;
        // one encoding per compute type, masked Hamming search per chain
        v[n++] = SV_SHARED;
    } else {
        if (!encoder_bucket(kind, x_type, ct, F, K))
            return -1;
        if (x_type == X_FP32 ? (ct == C_I8 || ct == C_I8S) : ct == C_F32)
            return -1;
        const int wi = width_index(x_type, F);
        const int width = x_type == X_FP32 ? kF32Widths[wi] : kIntWidths[wi];
        n = encoder_variants(ct, x_type, width, encoder_kt(kind == KK_ENCODE ? M_ENCODE : M_CLASSIFY, K),
                             kind == KK_CLASSIFY, v);
        if (n == 0)   // no kernel of this shape takes the pair
            return -1;
    }
    for (int i = 0; i < n && i < cap; ++i)
        out[i] = v[i];
    return n;
}

bool tile_compiled(int kind, int x_type, int ct, int F, int K, int variant)
{
    int v[8];
    const int n = tile_variants(kind, x_type, ct, F, K, v, 8);
    if (variant == 0)
        return n > 0;
    for (int i = 0; i < n; ++i)
        if (v[i] == variant)
            return true;
    return false;
}

}  // namespace hdc
