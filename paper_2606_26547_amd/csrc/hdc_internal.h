// Internal declarations shared by the HIP kernel sources and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hdc.h"

namespace hdc {

// Encoding compute type of a kernel instantiation.  C_FP8S is E4M3 on
// integer features split into a multiple of 16 and a remainder in [0, 16)
// (both exact in E4M3), two MFMAs per projection fragment.  C_I8S and
// C_FP8H are the int8 and E4M3 paths on the shifted projection p + 1 in
// {0, 2} (byte features, direct staging only): their kernels are the int8
// and E4M3 ones with EncodeArgs::poff set.
enum Compute : int { C_I8 = 0, C_BF16 = 1, C_FP8 = 2, C_F32 = 3, C_FP8S = 4, C_I8S = 5, C_FP8H = 6 };
constexpr int kComputeTypes = 7;

// Feature storage type.
enum XType : int { X_INT8 = 0, X_UINT8 = 1, X_FP32 = 2 };

// Operands of one encode / classify launch.  Dimension j of the launch is
// dimension s0 + j*stride of the projection, for j < nd.
struct EncodeArgs {
    const void *X;
    int x_type;            // XType
    int64_t n;
    int32_t F;
    int64_t ldx;           // elements
    const int8_t *P;
    int64_t ldp;           // bytes (= elements)
    int32_t s0, stride, nd;
    // encode mode: packed output, viewed as uint32 halves of the words
    uint32_t *H32;
    int64_t ldh32;         // row pitch in uint32
    // classify mode
    const int8_t *ctab;    // class operand table, [nchunk][KT][64 lanes][16 B]
    const int32_t *cpop;   // [KT*32] count of -1 elements of each class over S
    int32_t K;
    int32_t *labels;       // [n]
    int32_t *dists;        // [n][K] or null
    // dimension splits: a launch whose query blocks cannot fill the device
    // spreads the dimension list over gridDim.y workgroups per query block
    // (at most max_split; 0 or 1 = none).  Classify partials go to
    // part[split][K][n] (int32), then a small kernel takes the argmin.
    int32_t max_split;
    int32_t *part;
    int32_t nsplit;        // set by the launch: the splits it uses (1 = none)
    // 1: P holds the shifted weights p + 1 in {0, 2}; every accumulator
    // starts from minus the query's feature sum, so that it ends at the
    // same y as on the +-1 weights (int8 path, direct staging)
    int32_t poff;
};

// Dimension splits of an encoder launch with `blocks` query blocks over nd
// dimensions: as many as keep blocks * splits within `target` workgroups
// (the device's resident workgroups for the kernel: one round, no tail),
// each split at least kSplitMinUnits whole 64-dimension words, at most `cap`
// (1 = no split).  The kernel maps split z of Z to words [z*per, (z+1)*per)
// with per = split_units(nd, Z) = ceil(words / Z); the count returned is
// ceil(words / per), so that no split is empty.
constexpr int kSplitMinUnits = 4;
constexpr int kQpbMax = 256;        // most queries per encoder workgroup (any variant)
constexpr int kSplitTargetMax = 512;   // two resident workgroups per CU at most
__host__ __device__ inline int split_count(int64_t blocks, int nd, int cap, int target)
{
    const int units = (nd + 63) / 64;
    if (blocks <= 0 || 2 * blocks > target || units < 2 * kSplitMinUnits || cap < 2)
        return 1;
    int64_t z = target / blocks;
    const int zmax = units / kSplitMinUnits;
    z = z < zmax ? z : zmax;
    z = z < cap ? z : cap;
    const int per = (int)((units + z - 1) / z);
    return (units + per - 1) / per;
}
__host__ __device__ inline int split_units(int nd, int Z) { return ((nd + 63) / 64 + Z - 1) / Z; }

// Mode of the encode kernel.
enum Mode : int { M_ENCODE = 0, M_CLASSIFY = 1 };

// Kernel shape of one encode / classify launch (TileVariant; 0 = the
// built-in rule).
struct Tile {
    int variant;
};


constexpr int kDimChunk = 32;       // dimensions per MFMA row tile / LDS chunk
constexpr int kWaves = 4;           // waves per workgroup of the encoder
constexpr int kMaxF = 1024;
constexpr int kMaxFFloat = 256;
constexpr int kMaxK = 128;
constexpr int kMaxConfigs = 4096;
// The prepared searches address a workgroup's query rows with 32-bit byte
// offsets from its first row (at most 256 rows).
constexpr int64_t kMaxPreparedLdq = 1 << 20;
// Level-ID encoding keeps a window of every identity and level hypervector
// in LDS.
constexpr int kMaxLevelIdF = 1024;
constexpr int kMaxLevels = 1024;

inline int class_tiles(int K) { return (K + 31) / 32 <= 1 ? 1 : ((K + 31) / 32 <= 2 ? 2 : 4); }
inline int64_t chunks(int nd) { return (nd + kDimChunk - 1) / kDimChunk; }
// The fused classifier's class operand covers a whole number of every
// chunk width it is read in (2 and 3 tiles of 32: a multiple of kMaxRT
// tiles); rows past the dimension count are 0.
constexpr int kMaxRT = 6;
inline int64_t table_chunks(int nd) { return (chunks(nd) + kMaxRT - 1) / kMaxRT * kMaxRT; }
inline size_t class_table_bytes(int nd, int K) { return (size_t)table_chunks(nd) * class_tiles(K) * 1024; }

// Tile variants of the encoder: direct-to-LDS staging of the projection
// with two query tiles x two row tiles per wave or one of each (int8
// features on the int8 path), or register staging with one or two query
// tiles per wave.
enum TileVariant : int { TV_AUTO = 0, TV_DMA_2X2 = 1, TV_DMA_1X1 = 2, TV_REG_QT1 = 3, TV_REG_QT2 = 4,
                         TV_DMA_2X3 = 5 };
// Tile variants of the configuration sweep (per configuration): work items of
// 128 queries (one query tile per wave) or of 256 (int8 slots with two query
// tiles per wave where the registers allow, other slots in two passes), or of
// 256 with int8-feature int8 slots on the direct-staged 2x2 body; or shared:
// the configurations of one compute type take their Hamming distances from
// one encoding of the union of their dimension sets.
enum SweepVariant : int { SV_AUTO = 0, SV_ITEM128 = 1, SV_ITEM256 = 2, SV_ITEM256_DMA = 3, SV_SHARED = 4 };
enum KernelKind : int { KK_ENCODE = 0, KK_CLASSIFY = 1, KK_SWEEP = 2 };

// Shape rules shared by the kernel templates and the variant listing.
// Direct staging with 2x2 tiles fits the registers up to 20 K steps and two
// class tiles.
constexpr bool big_tile(int ks, int kt) { return ks <= 20 && kt <= 2; }
// The classifier's 2x3 shape (two query tiles x three row tiles, chunks of
// 96 dimensions in a two-stage ring): one class tile.
constexpr bool big3_tile(int ks, int kt) { return ks <= 20 && kt == 1; }
// The shifted projection (C_I8S): the 2x2 / 2x3 shapes from 10 K steps (F >
// 256) up, which run one wave per SIMD and have registers to spare for the
// start values of their accumulators.
constexpr bool shift_tile(int ks, int kt) { return ks >= 10 && big_tile(ks, kt); }
// The E4M3 path on the shifted projection (C_FP8H): the direct-staged 2x2
// shape from 5 to 10 K steps of 64 features (256 < F <= 640), up to two
// class tiles.
constexpr bool shift8_tile(int ks, int kt) { return ks >= 5 && ks <= 10 && kt <= 2; }
// Two query tiles per wave fit beside the accumulators (register staging).
constexpr bool qt2_fits(int ct, int ks) { return (ct == C_I8 && ks <= 16) || (ct == C_F32 && ks <= 64); }
// K step (features per MFMA) of a compute type.
constexpr int kstep_of(int ct)
{
    return ct == C_I8 || ct == C_I8S ? 32 : (ct == C_FP8 || ct == C_FP8S || ct == C_FP8H) ? 64 : ct == C_BF16 ? 16 : 2;
}

// Compiled feature widths of the encoder (integer features / fp32
// features); a launch uses the smallest width >= F.
constexpr int kIntWidths[] = {64, 128, 192, 256, 320, 384, 512, 640, 832, 1024};
constexpr int kF32Widths[] = {64, 128, 256};
// Compiled feature widths of the sweep.
constexpr int kSweepWidths[] = {128, 256, 512, 640, 832, 1024};
int width_index(int x_type, int F);          // -1 if F is beyond the compiled widths
int sweep_width_index(int F);
// Class tiles a launch is compiled for.
inline int encoder_kt(int mode, int K) { return mode == M_ENCODE ? 1 : class_tiles(K); }
inline int sweep_kt(int K) { return K <= 32 ? 1 : 4; }

// Tile variants a bucket is compiled with (the built-in one first; -1 for a
// shape outside the compiled kernels), and whether a launch may name one.
int tile_variants(int kind, int x_type, int ct, int F, int K, int *out, int cap);
bool tile_compiled(int kind, int x_type, int ct, int F, int K, int variant);

hipError_t launch_encode(const EncodeArgs &a, int compute, int mode, Tile tile, hipStream_t st);
hipError_t launch_class_table(const uint64_t *C, int K, int64_t ldc, int s0, int stride, int nd,
                              int8_t *tab, int32_t *cpop, hipStream_t st);
hipError_t launch_class_popc(const uint64_t *C, int K, int64_t ldc, int s0, int stride, int nd, int KT,
                             int32_t *cpop, hipStream_t st);
size_t ham_workspace_bytes(int start, int end, int K);
hipError_t launch_ham_prepare(const uint64_t *C, int K, int64_t ldc, int start, int end, int stride, uint8_t *ws,
                              hipStream_t st);
hipError_t launch_ham_prepared(const uint64_t *Q, int64_t n, int64_t ldq, int K, int start, int end,
                               const uint8_t *ws, int32_t *argmin, int32_t *min_dist, int32_t *dists,
                               hipStream_t st);
size_t cos_workspace_bytes(int start, int end, int K);
hipError_t launch_cos_prepare(const int32_t *acc, int K, int64_t lda, int start, int end, int stride, uint8_t *ws,
                              hipStream_t st);
hipError_t launch_cos_prepared(const uint64_t *Q, int64_t n, int64_t ldq, int K, int start, int end,
                               const uint8_t *ws, int32_t *label, double *max_score, double *scores,
                               hipStream_t st);
hipError_t launch_hamming(const uint64_t *Q, int64_t n, int64_t ldq, const uint64_t *C, int K,
                          int64_t ldc, int start, int end, int stride, int32_t *argmin,
                          int32_t *min_dist, int32_t *dists, hipStream_t st);
// Bundling and retraining (hdc_bundle.hip): mode 0 bundle (accumulator in
// the workspace), 1 class accumulators, 2 one retraining epoch.
bool group_count_fits(int64_t n);
size_t group_count_ws_bytes(int mode, int64_t n, int nbits, int K);
// The no-allocation bundling entry point's device scratch (hdc_bundle.hip):
// its size, and its address on the current device (looked up on the first
// call per device).
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
hipError_t noalloc_scratch(void **out);
hipError_t launch_group_count(int mode, const uint64_t *H, int64_t n, int nbits, int64_t ldh, const int32_t *labels,
                              const int32_t *pred, int K, int32_t *acc, uint64_t *C, int64_t ldc, int32_t *counts,
                              int32_t *n_wrong, void *ws, hipStream_t st);
hipError_t launch_adc_argmax(const uint64_t *Q, int64_t n, int64_t ldq, const uint64_t *C, int K, int64_t ldc,
                             int start, int end, int stride, int res, int step, int floor_, int ceil_,
                             int32_t *label, int32_t *max_score, int32_t *scores, hipStream_t st);
hipError_t launch_shift_projection(const int8_t *P, int D, int F, int64_t ldp, bool e4m3, int8_t *out,
                                   int64_t ldo, hipStream_t st);
hipError_t launch_gather_cols(const void *X, int elem, int64_t n, int64_t ldx, int start, int stride, int nf,
                              void *Y, int64_t ldy, hipStream_t st);
hipError_t launch_level_quantize(const float *X, int64_t n, int F, int64_t ldx, const float *lo, const float *hi,
                                 int L, uint16_t *lev, int64_t ldl, hipStream_t st);
hipError_t launch_level_id(const uint16_t *lev, int64_t n, int F, int64_t ldl, const uint64_t *ID, int64_t ldid,
                           const uint64_t *LV, int L, int64_t ldlv, int D, uint64_t *H, int64_t ldh,
                           hipStream_t st);
size_t adc_workspace_bytes(int start, int end, int K);
hipError_t launch_adc_prepare(const uint64_t *C, int K, int64_t ldc, int start, int end, int stride, uint8_t *ws,
                              hipStream_t st);
hipError_t launch_adc_prepared(const uint64_t *Q, int64_t n, int64_t ldq, int K, int start, int end, int res,
                               int step, int floor_, int ceil_, const uint8_t *ws, int32_t *label,
                               int32_t *max_score, int32_t *scores, hipStream_t st);
hipError_t launch_convert(const void *X, int x_type, int64_t n, int F, int64_t ldx, int compute,
                          float *out, hipStream_t st);

// Persistent configuration sweep.
struct SweepArgs {
    const void *X;
    int x_type;
    int64_t n;
    int32_t F;
    int64_t ldx;
    const int32_t *truth;
    const int8_t *P;
    int64_t ldp;
    int32_t D;
    const uint64_t *C;
    int32_t K;
    int64_t ldc;
    const hdc_config *cfgs;   // host
    int32_t ncfg;
    hdc_config_result *out;   // host
    uint8_t *ws;
    size_t ws_bytes;
    int32_t max_wg;           // 0: fill the device
};
size_t sweep_workspace_bytes(int32_t ncfg, int32_t F, int32_t D, int32_t K);
hipError_t launch_sweep(const SweepArgs &a, hipStream_t st);

}  // namespace hdc
