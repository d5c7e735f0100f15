// Class bundling and retraining updates (Sec. 2.1: same-class hypervectors
// are aggregated into one class hypervector; Sec. 5: the retraining
// iterations of the apps), as one counting pipeline over the training
// hypervectors.
//
// Every call adds, for a list of (row, class, sign) entries, the bipolar
// value of each bit (+1 for bit 0, -1 for bit 1) times the sign into an int32
// accumulator acc[class][d]; the class hypervector bit is then (acc < 0), so
// a zero sum (a tie, or an empty class) gives +1.
//   bundle:      entries (i, labels[i], +1) for every row: acc is the
//                bipolar class sum, and acc < 0 is exactly 2*cnt > n_k.
//   class_acc:   the same entries, acc returned to the caller.
//   retrain:     for a mispredicted row, (i, labels[i], +1) and
//                (i, pred[i], -1), added onto the caller's acc.
//
// Pipeline (all device work, integer arithmetic only, so the result does not
// depend on the order in which rows are visited):
//   1. group the entries by (class, sign) into a row-index list: per-block
//      histograms, one scan, a scatter (one fused single-workgroup kernel
//      for small inputs; a small bundle does all three steps in one kernel,
//      k_bundle_small);
//   2. count: each workgroup takes a segment of up to R rows of one group
//      and a column tile of the hypervectors; every lane owns V dwords of
//      the row and counts the set bits of the rows it reads with bit-sliced
//      carry-save adders (sixteen rows folded per step, a vertical counter
//      above them), so the per-row cost is a few bitwise operations per
//      32 bits and no atomics; at the end each lane turns its counters into
//      per-dimension counts, the four waves add them in LDS, and the
//      workgroup adds sign * (rows - 2*count) into acc with one integer
//      atomic per dimension;
//   3. binarise acc into the class words (one ballot per 64 dimensions).
#include <mutex>

#include "hdc_device.h"

namespace hdc {

namespace {

constexpr int kGroupMax = 2 * kMaxK;   // groups: classes, or (class, sign) pairs
constexpr int kRowsPerThread = 16;     // rows per thread of a histogram / scatter block
constexpr int kBlockRows = 256 * kRowsPerThread;
constexpr int kSmallRowsPerThread = 8;
constexpr int kSmallRows = 1024 * kSmallRowsPerThread;   // one fused grouping workgroup up to here
constexpr int kPlanes = 8;             // vertical counter above the sixteens
constexpr int kMinSeg = 256, kMaxSeg = 8192;   // rows per count segment

enum GroupMode : int { GM_BUNDLE = 0, GM_CLASS_ACC = 1, GM_RETRAIN = 2 };

struct GroupArgs {
    const int32_t *labels;
    const int32_t *pred;       // retrain only
    int64_t n;
    int32_t K, G, mode, R;     // classes, groups, GroupMode, rows per segment
    int32_t B;                 // histogram blocks of kBlockRows rows
    int32_t *hist;             // [B][G] per-block group sizes
    int32_t *cursor;           // [G] next free list entry of each group
    int32_t *goff;             // [G + 1] first list entry of each group
    int32_t *segoff;           // [G + 1] first count segment of each group
    int32_t *idx;              // list of row indices, grouped
    int32_t *counts;           // [K] class sizes (bundle), may be null
    int32_t *n_wrong;          // retrain: mispredicted rows, may be null
    int32_t *zero;             // int32 array cleared before counting, may be null
    int64_t zero_count;
};

// Group keys of rows r0 + threadIdx.x + j * blockDim.x (j < RPT, rows below
// r1): k0 / k1 = -1 where a row has no (second) key.  Every load is issued
// before any key is used.
template <int RPT>
__device__ __forceinline__ void load_keys(const GroupArgs &a, int64_t r0, int64_t r1, int (&k0)[RPT],
                                          int (&k1)[RPT])
{
    int y[RPT], p[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int64_t i = r0 + threadIdx.x + (int64_t)j * blockDim.x;
        y[j] = i < r1 ? a.labels[i] : -1;
        p[j] = a.mode == GM_RETRAIN && i < r1 ? a.pred[i] : -1;
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const bool yok = y[j] >= 0 && y[j] < a.K;
        if (a.mode != GM_RETRAIN) {
            k0[j] = yok ? y[j] : -1;
            k1[j] = -1;
        } else {
            const bool w = yok && p[j] >= 0 && p[j] < a.K && p[j] != y[j];
            k0[j] = w ? 2 * y[j] : -1;
            k1[j] = w ? 2 * p[j] + 1 : -1;
        }
    }
}

template <int RPT>
__device__ __forceinline__ void hist_keys(const int (&k0)[RPT], const int (&k1)[RPT], int *lh)
{
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        if (k0[j] >= 0)
            atomicAdd(&lh[k0[j]], 1);
        if (k1[j] >= 0)
            atomicAdd(&lh[k1[j]], 1);
    }
}

template <int RPT>
__device__ __forceinline__ void scatter_keys(const GroupArgs &a, int64_t r0, const int (&k0)[RPT],
                                             const int (&k1)[RPT], int *lpos)
{
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int32_t i = (int32_t)(r0 + threadIdx.x + (int64_t)j * blockDim.x);
        if (k0[j] >= 0)
            a.idx[atomicAdd(&lpos[k0[j]], 1)] = i;
        if (k1[j] >= 0)
            a.idx[atomicAdd(&lpos[k1[j]], 1)] = i;
    }
}

// Exclusive prefix sums of two per-thread values over the block (at most
// 16 waves); `wt` is LDS of 2 * 16 ints.  Every thread must call it.
__device__ __forceinline__ void block_scan2(int v0, int v1, int *e0, int *e1, int *wt)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int s0 = v0, s1 = v1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u0 = __shfl_up(s0, o), u1 = __shfl_up(s1, o);
        if (lane >= o) {
            s0 += u0;
            s1 += u1;
        }
    }
    if (lane == 63) {
        wt[wave] = s0;
        wt[16 + wave] = s1;
    }
    __syncthreads();
    int b0 = 0, b1 = 0;
    for (int w = 0; w < wave && w < nw; ++w) {
        b0 += wt[w];
        b1 += wt[16 + w];
    }
    *e0 = b0 + s0 - v0;
    *e1 = b1 + s1 - v1;
    __syncthreads();
}

// Group sizes (tot, LDS) -> offsets of the groups and of their count
// segments, class sizes, mispredicted rows; each group's cursor (LDS and
// global, either may be null) starts at its first entry.  blockDim >= G.
__device__ void finish_groups(const GroupArgs &a, const int *tot, int *lcur, int *wt)
{
    const int g = threadIdx.x;
    const int ng = g < a.G ? tot[g] : 0;
    int e, sgo;
    block_scan2(ng, (ng + a.R - 1) / a.R, &e, &sgo, wt);
    if (g < a.G) {
        a.goff[g] = e;
        a.segoff[g] = sgo;
        if (a.cursor)
            a.cursor[g] = e;
        if (lcur)
            lcur[g] = e;
        if (a.counts)
            a.counts[g] = ng;
    }
    if (g == a.G - 1) {
        a.goff[a.G] = e + ng;
        a.segoff[a.G] = sgo + (ng + a.R - 1) / a.R;
    }
    if (a.mode == GM_RETRAIN && a.n_wrong) {   // mispredicted rows = entries of the (class, +) groups
        int v = g < a.G && !(g & 1) ? ng : 0, ex, dummy;
        block_scan2(v, 0, &ex, &dummy, wt);
        if (g == blockDim.x - 1)
            *a.n_wrong = ex + v;
    }
}

__device__ void zero_part(const GroupArgs &a, int64_t part, int64_t parts)
{
    for (int64_t i = part * blockDim.x + threadIdx.x; i < a.zero_count; i += parts * blockDim.x)
        a.zero[i] = 0;
}

// Small inputs: block 0 (1024 threads) histograms, scans and scatters all
// rows; the other blocks clear the accumulator.
__global__ __launch_bounds__(1024) void k_group_small(GroupArgs a)
{
    __shared__ int lh[kGroupMax], lpos[kGroupMax], wt[32];
    if (blockIdx.x > 0) {
        zero_part(a, blockIdx.x - 1, gridDim.x - 1);
        return;
    }
    for (int g = threadIdx.x; g < a.G; g += blockDim.x)
        lh[g] = 0;
    int k0[kSmallRowsPerThread], k1[kSmallRowsPerThread];
    load_keys<kSmallRowsPerThread>(a, 0, a.n, k0, k1);
    __syncthreads();
    hist_keys<kSmallRowsPerThread>(k0, k1, lh);
    __syncthreads();
    finish_groups(a, lh, lpos, wt);
    __syncthreads();
    scatter_keys<kSmallRowsPerThread>(a, 0, k0, k1, lpos);
}

// Large inputs, pass 1: per-block group sizes; the accumulator is cleared.
__global__ __launch_bounds__(256) void k_group_hist(GroupArgs a)
{
    __shared__ int lh[kGroupMax];
    for (int g = threadIdx.x; g < a.G; g += blockDim.x)
        lh[g] = 0;
    const int64_t r0 = (int64_t)blockIdx.x * kBlockRows;
    int k0[kRowsPerThread], k1[kRowsPerThread];
    load_keys<kRowsPerThread>(a, r0, r0 + kBlockRows < a.n ? r0 + kBlockRows : a.n, k0, k1);
    __syncthreads();
    hist_keys<kRowsPerThread>(k0, k1, lh);
    __syncthreads();
    for (int g = threadIdx.x; g < a.G; g += blockDim.x)
        a.hist[(int64_t)blockIdx.x * a.G + g] = lh[g];
    if (a.zero)
        zero_part(a, blockIdx.x, gridDim.x);
}

// Pass 2 (one block of 256 threads): group sizes and offsets.
__global__ __launch_bounds__(256) void k_group_scan(GroupArgs a)
{
    __shared__ int tot[kGroupMax], wt[32];
    for (int g = threadIdx.x; g < a.G; g += blockDim.x)
        tot[g] = 0;
    __syncthreads();
    const int64_t BG = (int64_t)a.B * a.G;
    for (int64_t i = threadIdx.x; i < BG; i += blockDim.x) {
        const int v = a.hist[i];
        if (v)
            atomicAdd(&tot[i % a.G], v);
    }
    __syncthreads();
    finish_groups(a, tot, nullptr, wt);
}

// Pass 3: each block reserves its part of every group (integer atomics on
// the group cursors: the order of blocks within a group is free, the counts
// do not depend on it) and scatters its rows.
__global__ __launch_bounds__(256) void k_group_scatter(GroupArgs a)
{
    __shared__ int lpos[kGroupMax];
    for (int g = threadIdx.x; g < a.G; g += blockDim.x) {
        const int h = a.hist[(int64_t)blockIdx.x * a.G + g];
        lpos[g] = h ? atomicAdd(&a.cursor[g], h) : 0;
    }
    const int64_t r0 = (int64_t)blockIdx.x * kBlockRows;
    int k0[kRowsPerThread], k1[kRowsPerThread];
    load_keys<kRowsPerThread>(a, r0, r0 + kBlockRows < a.n ? r0 + kBlockRows : a.n, k0, k1);
    __syncthreads();
    scatter_keys<kRowsPerThread>(a, r0, k0, k1, lpos);
}

// ---------------------------------------------------------------------------
// Counting.  Carry-save adder: h, l = the carry and sum bits of a + b + c.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void csa(uint32_t &h, uint32_t &l, uint32_t a, uint32_t b, uint32_t c)
{
    const uint32_t u = a ^ b;
    h = (u & c) | (~u & a);
    l = u ^ c;
}

template <int V>
struct BitCounters {
    uint32_t ones[V], twos[V], fours[V], eights[V], sp[kPlanes][V];
};

struct CountArgs {
    const uint32_t *H32;       // hypervector rows viewed as dwords
    int64_t ldh32;
    int32_t W32;               // dwords of a row that hold bits
    int32_t nbits, G, mode, R;
    const int32_t *goff, *segoff, *idx;
    int32_t *acc;              // [K][nbits] (row pitch nbits)
};

// Row indices of the sixteen rows r .. r + 15 (past `last`: the last row).
__device__ __forceinline__ void load_idx(const int32_t *idx, int64_t r, int64_t last, int32_t (&cur)[16])
{
#pragma unroll
    for (int u = 0; u < 16; ++u)
        cur[u] = idx[r + u <= last ? r + u : last];
}

template <int V>
__device__ __forceinline__ void load_rows(const uint32_t *H32, int64_t ldh32, const int32_t (&cur)[16], int coff,
                                          uint32_t (&x)[16][V])
{
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const uint32_t *row = H32 + (int64_t)cur[u] * ldh32;
        if (V == 2) {
            const uint2 q = *(const uint2 *)(row + coff);
            x[u][0] = q.x;
            x[u][V - 1] = q.y;
        } else {
            x[u][0] = row[coff];
        }
    }
}

// Adds rows r .. r + 15 (those up to `last`, in a column that holds bits)
// into the counters: fifteen carry-save adders fold the sixteen words into
// ones, twos, fours, eights and one word of sixteens, which enters the
// vertical counter.
template <int V>
__device__ __forceinline__ void add_rows(uint32_t (&x)[16][V], int64_t r, int64_t last, bool colok,
                                         BitCounters<V> &c)
{
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v)
            x[u][v] = colok && r + u <= last ? x[u][v] : 0u;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        uint32_t tA, tB, fA, fB, eA, eB, sx;
        csa(tA, c.ones[v], c.ones[v], x[0][v], x[1][v]);
        csa(tB, c.ones[v], c.ones[v], x[2][v], x[3][v]);
        csa(fA, c.twos[v], c.twos[v], tA, tB);
        csa(tA, c.ones[v], c.ones[v], x[4][v], x[5][v]);
        csa(tB, c.ones[v], c.ones[v], x[6][v], x[7][v]);
        csa(fB, c.twos[v], c.twos[v], tA, tB);
        csa(eA, c.fours[v], c.fours[v], fA, fB);
        csa(tA, c.ones[v], c.ones[v], x[8][v], x[9][v]);
        csa(tB, c.ones[v], c.ones[v], x[10][v], x[11][v]);
        csa(fA, c.twos[v], c.twos[v], tA, tB);
        csa(tA, c.ones[v], c.ones[v], x[12][v], x[13][v]);
        csa(tB, c.ones[v], c.ones[v], x[14][v], x[15][v]);
        csa(fB, c.twos[v], c.twos[v], tA, tB);
        csa(eB, c.fours[v], c.fours[v], fA, fB);
        csa(sx, c.eights[v], c.eights[v], eA, eB);
#pragma unroll
        for (int p = 0; p < kPlanes; ++p) {
            const uint32_t cy = c.sp[p][v] & sx;
            c.sp[p][v] ^= sx;
            sx = cy;
        }
    }
}

// Grid (segment, column tile).  Lane `lane` of every wave owns dwords
// [tile*64*V + lane*V, +V) of the rows; wave w takes rows
// begin + 16*(w + 4*j) .. +15 of the segment.
template <int V>
__global__ __launch_bounds__(256) void k_group_count(CountArgs a)
{
    __shared__ int lcnt[32 * V * 65];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int s = blockIdx.x, tile = blockIdx.y;
    const int nseg = a.segoff[a.G];
    if (s >= nseg)
        return;
    // the segment's group: the last g with segoff[g] <= s (empty groups
    // have segoff[g] == segoff[g + 1])
    int lo = 0, hi = a.G - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.segoff[mid] <= s)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int g = lo;
    const int64_t begin = (int64_t)a.goff[g] + (int64_t)(s - a.segoff[g]) * a.R;
    const int64_t gend = a.goff[g + 1];
    const int64_t end = begin + a.R < gend ? begin + a.R : gend;

    for (int i = t; i < 32 * V * 65; i += 256)
        lcnt[i] = 0;

    const int c0 = tile * 64 * V + lane * V;
    BitCounters<V> c;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        c.ones[v] = c.twos[v] = c.fours[v] = c.eights[v] = 0;
#pragma unroll
        for (int p = 0; p < kPlanes; ++p)
            c.sp[p][v] = 0;
    }
    // a column past the row's bits reads dword 0 of the row and counts it
    // as zero; so does a row past the segment's end (it reads the last row)
    const bool colok = c0 < a.W32;   // W32 is even: both dwords of a V = 2 lane agree
    const int coff = colok ? c0 : 0;
    const int64_t last = end - 1;
    // The wave index is uniform, so row indices live in scalar registers.
    // Two groups of sixteen rows are in flight: the next group's loads are
    // issued before the current group is counted, and its row indices one
    // group earlier still.
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    int64_t r = begin + 16 * wv;
    if (r < end) {
        int32_t ca[16], cb[16];
        uint32_t xa[16][V], xb[16][V];
        load_idx(a.idx, r, last, ca);
        load_rows<V>(a.H32, a.ldh32, ca, coff, xa);
        load_idx(a.idx, r + 64, last, cb);
        while (true) {
            const bool more = r + 64 < end;
            if (more)
                load_rows<V>(a.H32, a.ldh32, cb, coff, xb);
            if (r + 128 < end)
                load_idx(a.idx, r + 128, last, ca);
            add_rows<V>(xa, r, last, colok, c);
            r += 64;
            if (!more)
                break;
            const bool more2 = r + 64 < end;
            if (more2)
                load_rows<V>(a.H32, a.ldh32, ca, coff, xa);
            if (r + 128 < end)
                load_idx(a.idx, r + 128, last, cb);
            add_rows<V>(xb, r, last, colok, c);
            r += 64;
            if (!more2)
                break;
        }
    }
    __syncthreads();   // lcnt cleared
    // per-dimension counts of this wave's rows, added into LDS
#pragma unroll
    for (int v = 0; v < V; ++v)
        for (int j = 0; j < 32; ++j) {
            int cnt = (int)((c.ones[v] >> j) & 1u) + 2 * (int)((c.twos[v] >> j) & 1u) +
                      4 * (int)((c.fours[v] >> j) & 1u) + 8 * (int)((c.eights[v] >> j) & 1u);
            int hi16 = 0;
#pragma unroll
            for (int p = kPlanes - 1; p >= 0; --p)
                hi16 = 2 * hi16 + (int)((c.sp[p][v] >> j) & 1u);
            cnt += 16 * hi16;
            if (cnt)
                atomicAdd(&lcnt[(v * 32 + j) * 65 + lane], cnt);
        }
    __syncthreads();
    const int rows = (int)(end - begin);
    const int target = a.mode == GM_RETRAIN ? g >> 1 : g;
    const int sign = a.mode == GM_RETRAIN && (g & 1) ? -1 : 1;
    int32_t *accrow = a.acc + (int64_t)target * a.nbits;
    // thread e covers lane e / (32V), bit e % (32V): consecutive threads add
    // into consecutive dimensions
    for (int e = t; e < 64 * 32 * V; e += 256) {
        const int ln = e / (32 * V), jb = e % (32 * V);
        const int d = 32 * (tile * 64 * V + ln * V) + jb;
        if (d < a.nbits)
            atomicAdd(&accrow[d], sign * (rows - 2 * lcnt[jb * 65 + ln]));
    }
}

// Small bundles (n <= kSmallRows rows): one kernel instead of grouping,
// counting and binarising.  Workgroup (class k, column tile): the rows
// labelled k are listed in LDS (in any order: the counts are integers), the
// four waves count them as k_group_count does (sixteen rows per step, wave
// w from row 16w on, 64 rows apart), merge their per-dimension counts in
// LDS, and the tile's class words are written directly: bit d is set when
// more than half of the class's rows have it (acc < 0 with acc = rows -
// 2 * count); pad bits and an empty class give 0.
template <int V>
__global__ __launch_bounds__(256) void k_bundle_small(const uint32_t *__restrict__ H32, int64_t ldh32, int W32,
                                                      int nbits, const int32_t *__restrict__ labels, int n,
                                                      uint32_t *__restrict__ C32, int64_t ldc32,
                                                      int32_t *__restrict__ counts)
{
    __shared__ int32_t list[kSmallRows];
    __shared__ int lcnt[32 * V * 65];
    __shared__ int nrows;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int k = blockIdx.x, tile = blockIdx.y;
    if (t == 0)
        nrows = 0;
    for (int i = t; i < 32 * V * 65; i += 256)
        lcnt[i] = 0;
    __syncthreads();
#pragma unroll 4
    for (int i = t; i < n; i += 256)
        if (labels[i] == k)
            list[atomicAdd(&nrows, 1)] = i;
    __syncthreads();
    const int rows = nrows;
    const int c0 = tile * 64 * V + lane * V;
    BitCounters<V> c;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        c.ones[v] = c.twos[v] = c.fours[v] = c.eights[v] = 0;
#pragma unroll
        for (int p = 0; p < kPlanes; ++p)
            c.sp[p][v] = 0;
    }
    const bool colok = c0 < W32;
    const int coff = colok ? c0 : 0;
    const int64_t last = rows - 1;
    // the next sixteen rows' loads are in flight while the current ones
    // are counted
    auto fetch = [&](int r, uint32_t (&x)[16][V]) {
        int32_t cur[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            cur[u] = list[r + u <= last ? r + u : last];
        load_rows<V>(H32, ldh32, cur, coff, x);
    };
    int r = 16 * wave;
    if (r < rows) {
        uint32_t xa[16][V], xb[16][V];
        fetch(r, xa);
        while (true) {
            const bool more = r + 64 < rows;
            if (more)
                fetch(r + 64, xb);
            add_rows<V>(xa, r, last, colok, c);
            r += 64;
            if (!more)
                break;
            const bool more2 = r + 64 < rows;
            if (more2)
                fetch(r + 64, xa);
            add_rows<V>(xb, r, last, colok, c);
            r += 64;
            if (!more2)
                break;
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v)
        for (int j = 0; j < 32; ++j) {
            int cnt = (int)((c.ones[v] >> j) & 1u) + 2 * (int)((c.twos[v] >> j) & 1u) +
                      4 * (int)((c.fours[v] >> j) & 1u) + 8 * (int)((c.eights[v] >> j) & 1u);
            int hi16 = 0;
#pragma unroll
            for (int p = kPlanes - 1; p >= 0; --p)
                hi16 = 2 * hi16 + (int)((c.sp[p][v] >> j) & 1u);
            cnt += 16 * hi16;
            if (cnt)
                atomicAdd(&lcnt[(v * 32 + j) * 65 + lane], cnt);
        }
    __syncthreads();
    // thread e < 64V writes dword tile * 64V + e (lane e / V, part e % V)
    if (t < 64 * V) {
        const int dw = tile * 64 * V + t, ln = t / V, v = t % V;
        if (dw < W32) {
            uint32_t bits = 0;
            for (int j = 0; j < 32; ++j)
                if (32 * dw + j < nbits && 2 * lcnt[(v * 32 + j) * 65 + ln] > rows)
                    bits |= 1u << j;
            C32[(int64_t)k * ldc32 + dw] = bits;
        }
    }
    if (counts && tile == 0 && t == 0)
        counts[k] = rows;
}

// Class words from the accumulators: bit d of class k = (acc[k][d] < 0).
// One wave per word.
__global__ __launch_bounds__(256) void k_binarize(const int32_t *__restrict__ acc, int K, int nbits, int W,
                                                  uint64_t *__restrict__ C, int64_t ldc)
{
    const int64_t word = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (word >= (int64_t)K * W)
        return;
    const int k = (int)(word / W), w = (int)(word % W);
    const int d = 64 * w + lane;
    const bool neg = d < nbits && acc[(int64_t)k * nbits + d] < 0;
    const uint64_t bits = __ballot(neg);
    if (lane == 0)
        C[(int64_t)k * ldc + w] = bits;
}

struct Layout {
    int G, B, R, V, T;
    int64_t E, segs;
    size_t acc_off, hist_off, cursor_off, goff_off, segoff_off, idx_off, bytes;
};

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

Layout layout(int mode, int64_t n, int nbits, int K)
{
    Layout L;
    L.G = mode == GM_RETRAIN ? 2 * K : K;
    L.E = mode == GM_RETRAIN ? 2 * n : n;
    L.B = n <= kSmallRows ? 1 : (int)((n + kBlockRows - 1) / kBlockRows);
    const int W32 = 2 * ((nbits + 63) / 64);
    const int T1 = (W32 + 63) / 64, T2 = (W32 + 127) / 128;
    L.V = 2 * T2 == T1 ? 2 : 1;
    L.T = L.V == 2 ? T2 : T1;
    // about 2048 workgroups at the largest list the call can produce
    int64_t R = (L.E * L.T + 2047) / 2048;
    R = (R + 63) / 64 * 64;
    L.R = (int)(R < kMinSeg ? kMinSeg : R > kMaxSeg ? kMaxSeg : R);
    L.segs = (L.E + L.R - 1) / L.R + L.G;
    size_t off = 0;
    L.acc_off = off;
    if (mode == GM_BUNDLE)
        off = align256(off + (size_t)4 * K * nbits);
    L.hist_off = off;
    off = align256(off + (size_t)4 * L.B * L.G);
    L.cursor_off = off;
    off = align256(off + (size_t)4 * L.G);
    L.goff_off = off;
    off = align256(off + (size_t)4 * (L.G + 1));
    L.segoff_off = off;
    off = align256(off + (size_t)4 * (L.G + 1));
    L.idx_off = off;
    off = align256(off + (size_t)4 * (L.E > 0 ? L.E : 1));
    L.bytes = off;
    return L;
}

}  // namespace

// Scratch for callers that cannot allocate (hdc_bundle_noalloc): one array
// per device, held until the process ends.  Host code never uses the
// array's name as an address: the device address of each GPU's copy comes
// from hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];
}  // namespace

hipError_t noalloc_scratch(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kScratchDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Row indices and list offsets are int32; a retraining list holds up to 2n
// entries.
bool group_count_fits(int64_t n) { return n < ((int64_t)1 << 30); }

size_t group_count_ws_bytes(int mode, int64_t n, int nbits, int K) { return layout(mode, n, nbits, K).bytes; }

// mode: 0 bundle (acc in the workspace; counts and C written), 1 class_acc
// (acc cleared and written), 2 retrain (acc updated, n_wrong written).
hipError_t launch_group_count(int mode, const uint64_t *H, int64_t n, int nbits, int64_t ldh, const int32_t *labels,
                              const int32_t *pred, int K, int32_t *acc, uint64_t *C, int64_t ldc, int32_t *counts,
                              int32_t *n_wrong, void *ws, hipStream_t st)
{
    const Layout L = layout(mode, n, nbits, K);
    uint8_t *w8 = (uint8_t *)ws;
    if (mode == GM_BUNDLE)
        acc = (int32_t *)(w8 + L.acc_off);
    GroupArgs g;
    g.labels = labels;
    g.pred = pred;
    g.n = n;
    g.K = K;
    g.G = L.G;
    g.mode = mode;
    g.R = L.R;
    g.B = L.B;
    g.hist = (int32_t *)(w8 + L.hist_off);
    g.cursor = L.B == 1 ? nullptr : (int32_t *)(w8 + L.cursor_off);
    g.goff = (int32_t *)(w8 + L.goff_off);
    g.segoff = (int32_t *)(w8 + L.segoff_off);
    g.idx = (int32_t *)(w8 + L.idx_off);
    g.counts = mode == GM_BUNDLE ? counts : nullptr;
    g.n_wrong = mode == GM_RETRAIN ? n_wrong : nullptr;
    g.zero = mode == GM_RETRAIN ? nullptr : acc;
    g.zero_count = mode == GM_RETRAIN ? 0 : (int64_t)K * nbits;
    if (mode == GM_BUNDLE && n > 0 && n <= kSmallRows) {
        const dim3 grid((unsigned)K, (unsigned)L.T);
        const int W32 = 2 * ((nbits + 63) / 64);
        if (L.V == 2)
            hipLaunchKernelGGL(k_bundle_small<2>, grid, dim3(256), 0, st, (const uint32_t *)H, 2 * ldh, W32, nbits,
                               labels, (int)n, (uint32_t *)C, 2 * ldc, counts);
        else
            hipLaunchKernelGGL(k_bundle_small<1>, grid, dim3(256), 0, st, (const uint32_t *)H, 2 * ldh, W32, nbits,
                               labels, (int)n, (uint32_t *)C, 2 * ldc, counts);
        return hipGetLastError();
    }
    if (L.B == 1) {
        const int64_t zb = g.zero ? (g.zero_count + 1023) / 1024 : 0;
        hipLaunchKernelGGL(k_group_small, dim3((unsigned)(1 + (zb < 1024 ? zb : 1024))), dim3(1024), 0, st, g);
    } else {
        hipLaunchKernelGGL(k_group_hist, dim3((unsigned)L.B), dim3(256), 0, st, g);
        hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(256), 0, st, g);
        hipLaunchKernelGGL(k_group_scatter, dim3((unsigned)L.B), dim3(256), 0, st, g);
    }
    CountArgs c;
    c.H32 = (const uint32_t *)H;
    c.ldh32 = 2 * ldh;
    c.W32 = 2 * ((nbits + 63) / 64);
    c.nbits = nbits;
    c.G = L.G;
    c.mode = mode;
    c.R = L.R;
    c.goff = g.goff;
    c.segoff = g.segoff;
    c.idx = g.idx;
    c.acc = acc;
    if (n > 0) {
        const dim3 grid((unsigned)L.segs, (unsigned)L.T);
        if (L.V == 2)
            hipLaunchKernelGGL(k_group_count<2>, grid, dim3(256), 0, st, c);
        else
            hipLaunchKernelGGL(k_group_count<1>, grid, dim3(256), 0, st, c);
    }
    const int W = (nbits + 63) / 64;
    hipLaunchKernelGGL(k_binarize, dim3((unsigned)(((int64_t)K * W + 3) / 4)), dim3(256), 0, st, acc, K, nbits, W, C,
                       ldc);
    return hipGetLastError();
}

}  // namespace hdc
