// Bucketed segmented sort + pair pass: the fused SDM timestep on gfx950.
//
// Step 1 of the paper (Sec. 2.2, Sec. 3.2) orders each cell's live SDs by a
// random key (the GPU strategy the paper describes: a sort with random
// keys) and pairs neighbours; Steps 2-3 evaluate eq. (3), gamma and
// eqs. (4)-(6) per pair.  Four kernels:
//
//  k_tile    one workgroup per tile of T SD slots (coalesced reads of xi and
//            v): Step 0 liveness (xi > 0), Philox shuffle key, bucket =
//            (cell, top key bits); an LDS counting sort by bucket, then the
//            tile's records (id, 24 key bits and the bucket, xi, v) are
//            written contiguously through LDS staging, with the tile's
//            per-bucket offsets.  No global atomics except one per tile
//            (live total).
//  k_colsum  the global start rank of every bucket (hence of every group
//            and cell): the column sums of the tiles' exclusive bucket
//            offsets; and those offsets transposed to bucket-major order.
//  k_group   one workgroup per group of consecutive buckets: gathers the
//            group's run from every tile, sorts in LDS (counting sort by the
//            next key bits, then exact ranks by (key, s) in each
//            sub-bucket), keeps the sorted records in LDS, writes idx, and
//            evaluates the pairs, two adjacent ones per thread: probability,
//            gamma (one Philox block per two slots) and the collision update,
//            written back only for pairs that collide.  Groups are
//            independent; a pair straddling two groups leaves a seam record.
//  k_finish  the straddling pairs, the live count, and the per-launch
//            bookkeeping.
//
// A group with more records than its LDS capacity is sorted in global
// memory by a bitonic network instead (exact, only slower; for i.i.d. keys
// practically never taken).
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>

#include "sdm_internal.h"

namespace sdm {

constexpr int TILE_THREADS = 1024;
constexpr int TILE_EPT_MAX = 16;  // SD slots per tile thread (4, 8 or 16 per plan)
constexpr int TILE_FILL = 256;    // tiles that fill the GPU (one per CU)
constexpr int GROUP_THREADS = 512;
constexpr int GROUP_EPT_S = 7;       // records per group thread: the usual plans
constexpr int GROUP_EPT_L = 8;       // plans whose buckets hold more than GROUP_TARGET SDs
constexpr int MAXB = 32;             // buckets per group
constexpr int MAX_TILES = 2048;      // tiles per launch
constexpr int MAX_B = 16384;         // buckets per plan (LDS histogram)
constexpr int MAX_B_BATCH = 1 << 18; // batched plans (a tile histograms only its runs' buckets)
constexpr int TILE_LDS_BUDGET = 150 * 1024;
constexpr double BUCKET_TARGET = 1024.0;
constexpr double GROUP_TARGET = 3100.0;  // expected SDs per group of GROUP_EPT_S plans
constexpr uint32_t NO_BUCKET = 0xFFFFu;

__device__ __forceinline__ uint32_t load32_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ args
struct TileArgs {
    int mode;
    int64_t n_sd;
    const int64_t *n_live_in;
    const uint32_t *idx_in;
    const uint64_t *xi;
    const double *v;
    const int32_t *cell_id;
    int32_t n_cell;
    const double *u01;
    uint64_t seed;
    uint32_t run;
    uint32_t step;
    const uint32_t *step_dev;
    int key_shift;
    const int32_t *cell_h;
    const int32_t *cell_bucket_base;
    int32_t B;
    const uint32_t *seg_off;
    const uint32_t *seg_len;
    const int32_t *seg_run;
    uint16_t *tile_off;
    uint32_t tile_slots;   // SD slots of a tile (even, <= THREADS * EPT)
    const int32_t *tile_lb;      // batched plans: the tile's local bucket range
    const int32_t *tile_nb;
    const uint32_t *tile_loff;
    RecK *rec_k;           // list modes: (key, id)
    uint64_t *rec_f;       // fused mode records (8 B, RF_* layout)
    uint32_t chunk;        // 16-B records per LDS staging pass
    uint32_t *start_zero;  // bucket_start to clear for k_colsum's sums (or null)
    uint32_t *n_acc;
    uint32_t *err;
};

struct GroupArgs {
    int mode;
    int direct;                // one cell or groups of whole cells, dense tables,
                               // n_tiles <= group threads: bucket starts summed
                               // from tile_off (no k_colsum)
    const uint32_t *n_total;   // live SDs of the launch (the tiles' sum; direct)
    int32_t B;
    int32_t n_tiles;
    int32_t tile;
    int32_t n_cell;
    const int32_t *group_first;
    const int32_t *bucket_cell;
    const uint8_t *sub_bits;
    const int32_t *cell_h;
    const int32_t *cell_bucket_base;
    const uint16_t *tile_offT;  // [B+1][n_tiles] (dense plans)
    const uint16_t *tile_off;   // batched plans: local tables
    const int32_t *tile_lb;
    const int32_t *tile_nb;
    const uint32_t *tile_loff;
    const RecK *rec_k;
    const uint64_t *rec_f;
    const int32_t *cell_id;
    const uint32_t *bucket_start;
    uint32_t *cell_start;
    uint64_t *sk;
    uint32_t *ss;
    uint32_t *sb;
    int32_t group_cap;
    uint32_t *idx_out;
    uint64_t *xi;
    double *attr;
    int32_t n_attr;
    int64_t stride;
    double dt;
    const double *dv_cell;
    double dv;
    KernelDesc kern;
    const uint32_t *seg_off;
    const int32_t *seg_run;
    const int32_t *seg_kernel;
    const double *seg_dv;
    const KernelDesc *kernels;
    uint64_t seed;
    uint32_t run;
    uint32_t step;
    const uint32_t *step_dev;
    int slot_cell_local;
    uint64_t *counters;
    double *gamma_out;
    SeamRec *seam_open;
    SeamRec *seam_close;
    uint32_t *seam_state;
    uint32_t *group_tot;
    uint32_t *group_stats;  // [G][5] collision statistics per group
};

struct FinishArgs {
    int mode;
    int32_t G;
    int32_t n_cell;
    const SeamRec *seam_open;
    const SeamRec *seam_close;
    const uint32_t *seam_state;
    const uint32_t *group_tot;
    const uint32_t *group_stats;
    uint64_t *xi;
    double *attr;
    int32_t n_attr;
    int64_t stride;
    double dt;
    const double *dv_cell;
    double dv;
    KernelDesc kern;
    const uint32_t *seg_off;
    const int32_t *seg_run;
    const int32_t *seg_kernel;
    const double *seg_dv;
    const KernelDesc *kernels;
    uint64_t seed;
    uint32_t run;
    int slot_cell_local;
    uint64_t *counters;
    double *gamma_out;
    uint32_t *n_acc;
    uint32_t *cell_start;
    int64_t *n_live_out;
    uint32_t *step_advance;
};

// --------------------------------------------------------------- helpers
// Segment (run) containing SD slot s: largest r with seg_off[r] <= s.
__device__ __forceinline__ int find_seg(const uint32_t *seg_off, int n, uint32_t s)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg_off[mid] <= s)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Largest i in [0, n) with tab[i] <= x (tab ascending, tab[0] <= x).
__device__ __forceinline__ int upper_index(const uint32_t *tab, int n, uint32_t x)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Workgroups are dispatched to the eight XCDs in turn (workgroup i to XCD
// i mod 8), each with its own L2.  Group g's runs end in the cache lines
// where group g + 1's begin, so consecutive groups go to the same XCD: XCD x
// takes the x-th of eight contiguous ranges of groups, in order.  A
// bijection of [0, n).
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_local_index(int b, int n)
{
    const int x = b % N_XCD, i = b / N_XCD;
    const int per = n / N_XCD, rem = n % N_XCD;
    return x * per + min(x, rem) + i;
}

// Inclusive scan over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    return wave_scan_u32(v);
}

// Exclusive scan over THREADS values held one per thread; *total gets the
// sum.  One barrier: every wave adds up the wave totals before its own.  The
// caller puts a barrier between the return and the next write to scratch.
template <int THREADS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *scratch,
                                                         uint32_t *total)
{
    constexpr int W = THREADS / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t x = wave_scan_u32(v);
    if (lane == 63)
        scratch[wid] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t t = scratch[w];
        before += w < wid ? t : 0u;
        all += t;
    }
    *total = all;
    return before + x - v;
}

// In-place exclusive scan of an LDS array of n <= THREADS*PER entries;
// arr[n] receives the total.
template <int THREADS, int PER>
__device__ __forceinline__ void lds_exclusive_scan(uint32_t *arr, int n, uint32_t *scratch)
{
    uint32_t loc[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int idx = threadIdx.x * PER + i;
        loc[i] = idx < n ? arr[idx] : 0u;
        sum += loc[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan<THREADS>(sum, scratch, &total);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int idx = threadIdx.x * PER + i;
        if (idx < n)
            arr[idx] = run;
        run += loc[i];
    }
    if (threadIdx.x == 0)
        arr[n] = total;
    __syncthreads();
}

// In-place exclusive scan of arr[0..n) in LDS for large n; returns the total.
// Each wave takes a contiguous run of 64-entry rows and scans it a row at a
// time, so a wave's accesses cover 64 consecutive words (one per bank) rather
// than one word per lane a whole chunk apart.  The caller puts a barrier
// between the return and the next use of arr or scratch.
template <int THREADS>
__device__ __forceinline__ uint32_t lds_scan_rows(uint32_t *arr, int n, uint32_t *scratch)
{
    constexpr int W = THREADS / 64, U = 4;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int rows = (n + 63) >> 6;
    const int per = (rows + W - 1) / W;
    const int r0 = min(rows, wid * per), r1 = min(rows, r0 + per);
    uint32_t s = 0;
    for (int r = r0; r < r1; ++r) {
        const int i = r * 64 + lane;
        s += i < n ? arr[i] : 0u;
    }
    s = wave_scan_u32(s);
    if (lane == 63)
        scratch[wid] = s;
    __syncthreads();
    uint32_t run = 0, all = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t t = scratch[w];
        run += w < wid ? t : 0u;
        all += t;
    }
    for (int r = r0; r < r1; r += U) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = (r + u) * 64 + lane;
            v[u] = r + u < r1 && i < n ? arr[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = (r + u) * 64 + lane;
            const uint32_t inc = wave_scan_u32(v[u]);
            if (r + u < r1 && i < n)
                arr[i] = run + inc - v[u];
            run += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        }
    }
    return all;
}

// lds_exclusive_scan on 16-bit entries (every sum below 2^16).
template <int THREADS, int PER>
__device__ __forceinline__ void lds_exclusive_scan16(uint16_t *arr, int n, uint32_t *scratch)
{
    uint32_t loc[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int idx = threadIdx.x * PER + i;
        loc[i] = idx < n ? arr[idx] : 0u;
        sum += loc[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan<THREADS>(sum, scratch, &total);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int idx = threadIdx.x * PER + i;
        if (idx < n)
            arr[idx] = (uint16_t)run;
        run += loc[i];
    }
    if (threadIdx.x == 0)
        arr[n] = (uint16_t)total;
    __syncthreads();
}

// -------------------------------------------------------------- k_colsum
struct ScanArgs {
    const uint16_t *tile_off;
    uint16_t *tile_offT;     // [B+1][n_tiles] transposed copy for the groups
    int32_t n_tiles;
    int32_t B;
    uint32_t *bucket_start;  // [B+1]
};

// Global start rank of every bucket: bucket b starts after the records of
// buckets < b in every tile, i.e. at the sum over tiles of the tile's
// exclusive offset of b (column sums of tile_off; column B gives the live
// total).  One workgroup per 64 x 64 block of (tiles, buckets): coalesced
// row reads, the block transposed through LDS into tile_offT, partial column
// sums added into bucket_start (zeroed by the tile kernel when the tiles
// span more than one block).
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_colsum(ScanArgs a)
{
    constexpr int W = THREADS / 64;
    __shared__ uint16_t blk[64][66];  // [tile][bucket], rows padded against bank conflicts
    __shared__ uint32_t part[W][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c0 = blockIdx.x * 64, t0 = blockIdx.y * 64;
    const int64_t Bp = a.B + 1;
    const int c = c0 + lane;
    // all 64 / W rows of a wave in flight together: clamped addresses,
    // out-of-range entries dropped after the load
    uint32_t sum = 0;
    const int cc0 = min(c, a.B);
    uint16_t v[64 / W];
#pragma unroll
    for (int j = 0; j < 64 / W; ++j) {
        const int t = min(t0 + w + j * W, a.n_tiles - 1);
        v[j] = a.tile_off[t * Bp + cc0];
    }
#pragma unroll
    for (int j = 0; j < 64 / W; ++j) {
        const int i = w + j * W;
        const uint16_t x = (t0 + i < a.n_tiles && c <= a.B) ? v[j] : (uint16_t)0;
        blk[i][lane] = x;
        sum += x;
    }
    part[w][lane] = sum;
    __syncthreads();
    for (int j = w; j < 64; j += W) {
        const int cc = c0 + j, t = t0 + lane;
        if (cc <= a.B && t < a.n_tiles)
            a.tile_offT[(int64_t)cc * a.n_tiles + t] = blk[lane][j];
    }
    if (w == 0 && c <= a.B) {
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < W; ++i)
            s += part[i][lane];
        if (gridDim.y == 1)
            a.bucket_start[c] = s;
        else
            atomicAdd(&a.bucket_start[c], s);
    }
}

// Batched plans: a tile holds the SDs of a few consecutive runs, so its
// table covers only their buckets (lb .. lb + nb - 1, plus the total).
// Bucket b's start rank = the totals of the tiles wholly below b (an
// exclusive scan of the tile totals) plus the local offsets of b in the
// tiles that straddle it (bk_ta[b] .. bk_tc[b] - 1, a handful).
struct BatchScanArgs {
    const uint16_t *tile_off;
    const uint32_t *tile_loff;
    const int32_t *tile_lb;
    const int32_t *tile_nb;
    const int32_t *bk_ta;
    const int32_t *bk_tc;
    int32_t n_tiles;
    int32_t B;
    uint32_t *bucket_start;  // [B+1]
};

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_colsum_batch(BatchScanArgs a)
{
    __shared__ uint32_t tt[MAX_TILES + 1];
    __shared__ uint32_t red[THREADS / 64 + 1];
    const int tid = threadIdx.x;
    for (int t = tid; t < a.n_tiles; t += THREADS)
        tt[t] = a.tile_off[a.tile_loff[t] + (uint32_t)a.tile_nb[t]];
    __syncthreads();
    lds_exclusive_scan<THREADS, (MAX_TILES + THREADS - 1) / THREADS>(tt, a.n_tiles, red);
    for (int b = blockIdx.x * THREADS + tid; b <= a.B; b += gridDim.x * THREADS) {
        const int ta = a.bk_ta[b], tc = a.bk_tc[b];
        uint32_t sum = tt[ta];
        for (int t = ta; t < tc; ++t)
            sum += a.tile_off[a.tile_loff[t] + (uint32_t)(b - a.tile_lb[t])];
        a.bucket_start[b] = sum;
    }
}

// Exclusive offset of bucket b in tile t: the dense table, or a batched
// plan's local one (0 below the tile's buckets, its total above them).
template <class Args>
__device__ __forceinline__ uint32_t tile_bucket_off(const Args &a, int t, int b)
{
    if (!a.tile_lb)
        return a.tile_offT[(int64_t)b * a.n_tiles + t];
    const int lb = a.tile_lb[t], nb = a.tile_nb[t];
    const int i = b <= lb ? -1 : min(b - lb, nb);
    return i < 0 ? 0u : (uint32_t)a.tile_off[a.tile_loff[t] + (uint32_t)i];
}

// ---------------------------------------------------------------- k_tile
template <int THREADS, int EPT, bool LIST>
__global__ __launch_bounds__(THREADS) void k_tile(TileArgs a)
{
    constexpr int T = THREADS * EPT;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t scan_scratch[THREADS / 64 + 1];
    const int B = a.B;
    // this tile's buckets: all B, or (batched plans) those of its runs,
    // lb .. lb + NB - 1; hist[NB] receives the total
    const int lb = a.tile_lb ? a.tile_lb[blockIdx.x] : 0;
    const int NB = a.tile_lb ? a.tile_nb[blockIdx.x] : B;
    uint32_t *hist = reinterpret_cast<uint32_t *>(smem);
    const int hist_bytes = ((NB + 1) * 4 + 15) & ~15;
    uint64_t *stage = reinterpret_cast<uint64_t *>(smem + hist_bytes);
    const int tid = threadIdx.x;
    for (int i = tid; i <= NB; i += THREADS)
        hist[i] = 0;
    if (a.start_zero)
        for (int i = blockIdx.x * THREADS + tid; i <= B; i += gridDim.x * THREADS)
            a.start_zero[i] = 0;

    const uint32_t step = step_of(a.step, a.step_dev);
    const int64_t n_items = LIST ? *a.n_live_in : a.n_sd;
    // slots [2 pair0, lim) of the launch's n_items belong to this tile
    const uint32_t TS = a.tile_slots;
    const int64_t pair0 = (int64_t)blockIdx.x * (TS / 2);
    const int64_t lim = min(n_items, 2 * pair0 + (int64_t)TS);

    // batched runs (fused mode): the runs this tile's slots fall in, with
    // their offset, length, Philox run, key bits and first bucket, in LDS
    // (up to SEGTAB runs; more fall back to global lookups)
    constexpr int SEGTAB = 256;
    __shared__ uint32_t st_off[SEGTAB + 1];
    __shared__ uint32_t st_len[SEGTAB];
    __shared__ int32_t st_run[SEGTAB], st_h[SEGTAB], st_bb[SEGTAB];
    __shared__ int st_first, st_n;
    const bool segtab = !LIST && a.seg_off != nullptr;
    if (segtab) {
        if (tid == 0) {
            const int64_t last = n_items > 0 ? n_items - 1 : 0;
            const uint32_t s_lo = (uint32_t)min<int64_t>(2 * pair0, last);
            const uint32_t s_hi = (uint32_t)min<int64_t>(2 * pair0 + TS - 1, last);
            const int f = find_seg(a.seg_off, a.n_cell, s_lo);
            const int l = find_seg(a.seg_off, a.n_cell, s_hi);
            st_first = f;
            st_n = l - f + 1 <= SEGTAB ? l - f + 1 : 0;
        }
        __syncthreads();
        const int f = st_first, n = st_n;
        for (int i = tid; i < n; i += THREADS) {
            st_off[i] = a.seg_off[f + i];
            st_len[i] = a.seg_len[f + i];
            st_run[i] = a.seg_run[f + i];
            st_h[i] = a.cell_h[f + i];
            st_bb[i] = a.cell_bucket_base[f + i];
        }
        if (tid == 0 && n > 0)
            st_off[n] = a.seg_off[f + n];
    }
    __syncthreads();

    // list modes keep whole keys; the fused mode keeps 24 key bits and the
    // bucket's low 8 bits (the record's high word) and,
    // with up to 8 slots per thread (registers allow it), loads the volumes
    // together with xi
    constexpr bool EARLY_V = !LIST && EPT <= 8;
    uint64_t key[LIST ? EPT : 1];
    uint32_t k32[LIST ? 1 : EPT];
    double vv[LIST ? 1 : EPT];
    uint64_t xv[EPT];
    uint32_t bk[EPT];  // bucket (low 16 bits) | rank in tile (high 16 bits)
    uint32_t sid[LIST ? EPT : 1];
    const int seg_n = segtab ? st_n : 0;

    // fused mode, up to 8 slots per thread (small launches, latency bound):
    // every slot pair's loads (xi, v, cell ids) are issued before any of
    // them is used, from clamped addresses, so that they are all in flight
    // together; the odd last slot of the launch is read on its own below.
    // With 16 slots per thread each pair is loaded where it is used (all
    // loaded up front measured slower: the tile kernel is issue-bound there).
    constexpr bool PRELOAD = !LIST && EPT <= 8;
    constexpr bool EARLY_CID = PRELOAD;
    uint32_t cid[EARLY_CID ? EPT : 1];
    if (PRELOAD && n_items >= 2) {
#pragma unroll
        for (int k = 0; k < EPT / 2; ++k) {
            const int64_t i0 = 2 * (pair0 + (int64_t)k * THREADS + tid);
            const int64_t ia = i0 + 1 < lim ? i0 : 0;
            const ulonglong2 xx = *reinterpret_cast<const ulonglong2 *>(a.xi + ia);
            xv[2 * k] = xx.x;
            xv[2 * k + 1] = xx.y;
            if (EARLY_V) {
                const double2 v2 = *reinterpret_cast<const double2 *>(a.v + ia);
                vv[2 * k] = v2.x;
                vv[2 * k + 1] = v2.y;
            }
            if (EARLY_CID && a.cell_id) {
                cid[2 * k] = (uint32_t)a.cell_id[ia];
                cid[2 * k + 1] = (uint32_t)a.cell_id[ia + 1];
            }
        }
    }

    int ti_prev = 0;  // the run of this thread's previous slot pair (LDS table row)
#pragma unroll
    for (int k = 0; k < EPT / 2; ++k) {
        const int64_t p = pair0 + (int64_t)k * THREADS + tid;
        const int64_t i0 = 2 * p;
        uint32_t s[2];
        bool live[2];
        int32_t cell[2];
        uint64_t x[2] = {0, 0};
        if (!LIST) {
            s[0] = (uint32_t)i0;
            s[1] = (uint32_t)(i0 + 1);
            double v[2] = {0.0, 0.0};
            if (i0 + 1 < lim && PRELOAD) {
                x[0] = xv[2 * k];
                x[1] = xv[2 * k + 1];
                if (EARLY_V) {
                    v[0] = vv[2 * k];
                    v[1] = vv[2 * k + 1];
                }
            } else if (i0 + 1 < lim) {
                const ulonglong2 xx = *reinterpret_cast<const ulonglong2 *>(a.xi + i0);
                x[0] = xx.x;
                x[1] = xx.y;
                if (EARLY_V) {
                    const double2 v2 = *reinterpret_cast<const double2 *>(a.v + i0);
                    v[0] = v2.x;
                    v[1] = v2.y;
                }
            } else if (i0 < lim) {
                x[0] = a.xi[i0];
                if (EARLY_V)
                    v[0] = a.v[i0];
            }
            if (EARLY_V) {
                vv[2 * k] = v[0];
                vv[2 * k + 1] = v[1];
            }
            live[0] = x[0] > 0;
            live[1] = x[1] > 0;
        } else {
            live[0] = i0 < lim;
            live[1] = i0 + 1 < lim;
            s[0] = live[0] ? a.idx_in[i0] : 0;
            s[1] = live[1] ? a.idx_in[i0 + 1] : 0;
        }
        int seg = 0;
        int ti = -1;  // the run's row in the LDS table
        if (seg_n > 0) {
            // the two slots of a pair share a run (runs start at even slots);
            // slots past a run's length (alignment padding) belong to none
            // a thread's slots grow with k: search on from its last run
            // (one LDS read while the run goes on)
            if (ti_prev + 1 < seg_n && st_off[ti_prev + 1] <= s[0])
                ti_prev += 1 + upper_index(st_off + ti_prev + 1, seg_n - ti_prev - 1, s[0]);
            ti = ti_prev;
            seg = st_first + ti;
            cell[0] = cell[1] = seg;
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (s[e] - st_off[ti] >= st_len[ti])
                    live[e] = false;
        } else if (a.seg_off) {
            // batched runs: slots past a run's length (alignment padding)
            // belong to no run
            seg = find_seg(a.seg_off, a.n_cell, s[0]);
            cell[0] = cell[1] = seg;
            if (LIST)
                cell[1] = find_seg(a.seg_off, a.n_cell, s[1]);
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (s[e] - a.seg_off[cell[e]] >= a.seg_len[cell[e]])
                    live[e] = false;
        } else if (EARLY_CID && i0 + 1 < lim) {
#pragma unroll
            for (int e = 0; e < 2; ++e)
                cell[e] = (a.cell_id && live[e]) ? (int32_t)cid[2 * k + e] : 0;
        } else {
#pragma unroll
            for (int e = 0; e < 2; ++e)
                cell[e] = (a.cell_id && live[e]) ? a.cell_id[s[e]] : 0;
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (live[e] && (cell[e] < 0 || cell[e] >= a.n_cell)) {
                atomicOr(a.err, 1u);
                live[e] = false;
            }
        }
        uint64_t kk[2] = {0, 0};
        if (a.mode == MODE_CELLSORT) {
            kk[0] = (uint64_t)i0 << a.key_shift;
            kk[1] = (uint64_t)(i0 + 1) << a.key_shift;
        } else if (a.u01) {
#pragma unroll
            for (int e = 0; e < 2; ++e)
                kk[e] = live[e] ? uniform_to_key(a.u01[s[e]]) : 0;
        } else if (!LIST) {
            if (live[0] || live[1]) {
                uint32_t run = a.run;
                uint64_t lp = (uint64_t)p;
                if (ti >= 0) {
                    run = (uint32_t)st_run[ti];
                    lp = (uint64_t)p - (st_off[ti] >> 1);
                } else if (a.seg_off) {
                    run = (uint32_t)a.seg_run[seg];
                    lp = (uint64_t)p - (a.seg_off[seg] >> 1);
                }
                const WordPair w = philox_words(a.seed, run, step, SDM_STREAM_SHUFFLE, lp);
                kk[0] = w.even >> 11;
                kk[1] = w.odd >> 11;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (live[e])
                    kk[e] = philox_word(a.seed, a.run, step, SDM_STREAM_SHUFFLE, s[e]) >> 11;
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int j = 2 * k + e;
            if (LIST)
                key[j] = kk[e];
            else
                k32[j] = 0;
            xv[j] = x[e];
            if (LIST)
                sid[j] = s[e];
            bk[j] = NO_BUCKET;
            if (live[e]) {
                const int h = ti >= 0 ? st_h[ti] : a.cell_h[cell[e]];
                const uint32_t bb =
                    (uint32_t)(ti >= 0 ? st_bb[ti] : a.cell_bucket_base[cell[e]]);
                const uint32_t b = bb + (h ? (uint32_t)(kk[e] >> (53 - h)) : 0u);
                const uint32_t r = atomicAdd(&hist[b - (uint32_t)lb], 1u);
                bk[j] = (b - (uint32_t)lb) | (r << 16);
                if (!LIST)  // the 24 key bits below the bucket's, and the bucket mod 32
                    k32[j] = ((uint32_t)(kk[e] >> (29 - h)) & 0xFFFFFFu) | ((b & 31u) << 24);
            }
        }
    }
    __syncthreads();
    // exclusive bucket offsets of this tile
    {
        const uint32_t total = lds_scan_rows<THREADS>(hist, NB, scan_scratch);
        if (tid == 0) {
            hist[NB] = total;
            if (total)
                atomicAdd(&a.n_acc[0], total);
        }
        __syncthreads();
    }
    uint16_t *toff = a.tile_off + (a.tile_lb ? (int64_t)a.tile_loff[blockIdx.x]
                                             : (int64_t)blockIdx.x * (B + 1));
    for (int b = tid; b <= NB; b += THREADS)
        toff[b] = (uint16_t)hist[b];
    const uint32_t total = hist[NB];
    uint32_t pos[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint32_t b = bk[j] & 0xFFFFu;
        pos[j] = b == NO_BUCKET ? 0xFFFFFFFFu : hist[b] + (bk[j] >> 16);
    }
    // staged, coalesced write-out of the tile's records in bucket order.
    // Fused mode: one 24-B record (id, 24 key bits and the bucket, xi, v);
    // list modes: (key, id).  Passes of a.chunk 16-B records.
    const int64_t rbase = (int64_t)blockIdx.x * TS;
    const uint32_t CH = a.chunk;
    if (LIST) {  // the list modes (the fused step always runs LIST = false)
        RecK *stk = reinterpret_cast<RecK *>(stage);
        for (uint32_t c0 = 0; c0 < total; c0 += CH) {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                if (pos[j] - c0 < CH) {  // (pos = 0xFFFFFFFF never lands in a pass)
                    RecK r;
                    r.key = key[j];
                    r.s = LIST ? sid[j]
                               : (uint32_t)(2 * (pair0 + (int64_t)(j >> 1) * THREADS + tid) +
                                            (j & 1));
                    r.pad = 0;
                    stk[pos[j] - c0] = r;
                }
            }
            __syncthreads();
            const uint32_t n = min(CH, total - c0);
            const uint4 *src = reinterpret_cast<const uint4 *>(stk);
            uint4 *dst = reinterpret_cast<uint4 *>(a.rec_k + rbase + c0);
            for (uint32_t i = tid; i < n; i += THREADS)
                dst[i] = src[i];
            __syncthreads();
        }
        return;
    }
    if (!EARLY_V) {
        // volumes, read now as coalesced pairs
#pragma unroll
        for (int k = 0; k < EPT / 2; ++k) {
            const int64_t i0 = 2 * (pair0 + (int64_t)k * THREADS + tid);
            double v0 = 0.0, v1 = 0.0;
            if (pos[2 * k] != 0xFFFFFFFFu || pos[2 * k + 1] != 0xFFFFFFFFu) {
                if (i0 + 1 < lim) {
                    const double2 v2 = *reinterpret_cast<const double2 *>(a.v + i0);
                    v0 = v2.x;
                    v1 = v2.y;
                } else {
                    v0 = a.v[i0];
                }
            }
            vv[2 * k] = v0;
            vv[2 * k + 1] = v1;
        }
    }
    // 8-B records per pass: slot in the tile, bucket mod 32, 24 key bits,
    // the bound codes of xi and v
    uint64_t *sta = stage;
    const uint32_t CHF = 2u * CH;
    for (uint32_t c0 = 0; c0 < total; c0 += CHF) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (pos[j] - c0 < CHF) {
                const uint32_t local = 2u * ((uint32_t)(j >> 1) * THREADS + (uint32_t)tid) +
                                       (uint32_t)(j & 1);
                const uint32_t codes = sd_codes(xv[j], vv[j]);
                sta[pos[j] - c0] = (uint64_t)local |
                                   ((uint64_t)(k32[j] >> 24) << RF_BKT_SHIFT) |
                                   ((uint64_t)(k32[j] & 0xFFFFFFu) << RF_KEY_SHIFT) |
                                   ((uint64_t)codes << RF_XC_SHIFT);
            }
        }
        __syncthreads();
        const uint32_t n = min(CHF, total - c0);
        uint64_t *dst = a.rec_f + rbase + c0;
        const uint4 *src4 = reinterpret_cast<const uint4 *>(sta);
        uint4 *dst4 = reinterpret_cast<uint4 *>(dst);
        for (uint32_t i = tid; i < n / 2; i += THREADS)
            dst4[i] = src4[i];
        if ((n & 1u) && tid == 0)
            dst[n - 1] = sta[n - 1];
        __syncthreads();
    }
}

// ------------------------------------------------------- pair evaluation
// Per-cell constants of eq. (3) and of the gamma draw.
struct PairCtx {
    double norm;         // (dt / dV_c) * F(n_c)
    int32_t kid;         // kernel id
    int32_t kidx;        // the cell's entry of the batch kernel table
    double kp;           // kernel parameter p[0]
    uint32_t run;
    uint32_t slot_base;  // rank from which slots are numbered
    uint32_t gbase;      // offset of the run's slots in gamma_out
};

// A kernel argument's value as an opaque uniform register (read back from
// the first lane).  Where a value may come either from a kernel argument or
// from a table in memory, this keeps the compiler from merging the two
// loads into one through a private copy of the argument (a scratch store by
// every thread).
__device__ __forceinline__ double arg_value(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ int32_t arg_value(int32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ const double *arg_value(const double *p)
{
    const uint64_t u = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (const double *)(((uint64_t)hi << 32) | lo);
}

// The single-kernel descriptor with every field an opaque uniform value.
__device__ __forceinline__ KernelDesc arg_value(const KernelDesc &k)
{
    KernelDesc d;
    d.id = arg_value(k.id);
    d.reserved = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        d.p[i] = arg_value(k.p[i]);
    d.table = arg_value(k.table);
    return d;
}

template <class Args>
__device__ __forceinline__ PairCtx pair_ctx(const Args &a, int32_t c, uint32_t cs, uint32_t n_c)
{
    PairCtx pc;
    double dvc;
    if (a.seg_run) {
        dvc = a.seg_dv[c];
        const int ki = a.seg_kernel[c];
        pc.kid = a.kernels[ki].id;
        pc.kidx = ki;
        pc.kp = a.kernels[ki].p[0];
        pc.run = (uint32_t)a.seg_run[c];
        pc.gbase = a.seg_off[c] >> 1;
    } else {
        dvc = a.dv_cell ? a.dv_cell[c] : arg_value(a.dv);
        pc.kid = arg_value(a.kern.id);
        pc.kidx = 0;
        pc.kp = arg_value(a.kern.p[0]);
        pc.run = a.run;
        pc.gbase = 0;
    }
    pc.norm = (a.dt / dvc) * (double)pair_scale((uint64_t)n_c);
    pc.slot_base = a.slot_cell_local ? cs : 0u;
    return pc;
}

// p of eq. (3) in the order kernel, times max xi, times (dt/dV) F(n).  The
// kernel's whole descriptor is read only for tabulated kernels (their table
// and grid); the others need p[0] alone.
template <class Args>
__device__ __forceinline__ double pair_prob(const Args &a, const PairCtx &pc, uint64_t xa,
                                            double va, uint64_t xb, double vb)
{
    KernelDesc kd;
    if (pc.kid == KERNEL_TABULATED) {
        if (a.seg_run)
            kd = a.kernels[pc.kidx];
        else
            kd = arg_value(a.kern);
    } else {
        kd.id = pc.kid;
        kd.reserved = 0;
        kd.p[0] = pc.kp;
        kd.p[1] = kd.p[2] = kd.p[3] = 0.0;
        kd.table = nullptr;
    }
    const double ak = kernel_value(kd, va, vb);
    const uint64_t xm = xa > xb ? xa : xb;
    return (ak * (double)xm) * pc.norm;
}

// Upper bound of p from the two SDs' codes (xi code | volume code << 8);
// +inf where the cell's factors are not all nonnegative.
__device__ __forceinline__ double pair_bound(const PairCtx &pc, uint32_t ca, uint32_t cb)
{
    if (!(pc.kp >= 0.0 && pc.norm >= 0.0))
        return __longlong_as_double(0x7FF0000000000000ll);
    const double a = kernel_bound(pc.kid, pc.kp, vcode_decode(ca >> 8), vcode_decode(cb >> 8));
    const double X = xcode_decode(max(ca & 255u, cb & 255u));
    return ((a * X) * pc.norm) * (1.0 + 0x1p-9);
}

template <class Args>
__device__ __forceinline__ void finish_pair(const Args &a, const PairCtx &pc, uint32_t q,
                                            double p, double phi, uint32_t sa, uint64_t xa,
                                            uint32_t sbb, uint64_t xb, Stats &st)
{
    const double gamma = ceil(p - phi);
    if (a.gamma_out)
        a.gamma_out[pc.gbase + q] = gamma;
    const Collision col = collide(xa, xb, gamma, st);
    if (col.g)
        apply_collision(col, sa, sbb, a.xi, a.attr, a.n_attr, a.stride);
}

// finish_pair with the pair's volumes at hand (the group kernel's records).
template <class Args>
__device__ __forceinline__ void finish_pair_v(const Args &a, const PairCtx &pc, uint32_t q,
                                              double p, double phi, uint32_t sa, uint64_t xa,
                                              double va, uint32_t sbb, uint64_t xb, double vb,
                                              Stats &st)
{
    const double gamma = ceil(p - phi);
    if (a.gamma_out)
        a.gamma_out[pc.gbase + q] = gamma;
    const Collision col = collide(xa, xb, gamma, st);
    if (col.g)
        apply_collision_v(col, sa, sbb, va, vb, a.xi, a.attr, a.n_attr, a.stride);
}

// Per-local-bucket tables of a group, in LDS.
struct GroupTabs {
    uint32_t *off;     // [nb+1] local offset of each bucket
    uint32_t *cs;      // [nb] rank of the first SD of the bucket's cell
    uint32_t *n;       // [nb] live SDs in the bucket's cell
    PairCtx *pc;       // [nb] per-cell constants (fused mode)
};

// Per-group collision statistics into the group's row (summed by k_finish).
template <int THREADS>
__device__ __forceinline__ void store_group_stats(const GroupArgs &a, int g, const Stats &st,
                                                  uint32_t *red)
{
    constexpr int W = THREADS / 64;
    const int tid = threadIdx.x;
    uint32_t v[5] = {st.pairs, st.coll, st.capped, st.zeroed, st.ge2};
#pragma unroll
    for (int i = 0; i < 5; ++i)
        v[i] = wave_scan_u32(v[i]);  // lane 63: the wave's sum
    if ((tid & 63) == 63) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
            red[i * W + (tid >> 6)] = v[i];
    }
    __syncthreads();
    if (tid < 5) {
        uint32_t sum = 0;
        for (int w = 0; w < W; ++w)
            sum += red[tid * W + w];
        a.group_stats[g * 5 + tid] = sum;
    }
}

// Output phase of the global-memory path.  Get gives
// s / xi / v at local position f.
template <int THREADS, class Get>
__device__ void group_outputs(const GroupArgs &a, int g, int b0, int nb, uint32_t tot,
                              uint32_t rank0, const GroupTabs &T, const Get &get, uint32_t *red,
                              uint32_t *s_misc, uint32_t *opl)
{
    const int tid = threadIdx.x;
    for (uint32_t f = tid; f < tot; f += THREADS)
        a.idx_out[rank0 + f] = get.s(f);
    if (a.mode != MODE_FUSED)
        return;
    const uint32_t step = step_of(a.step, a.step_dev);
    Stats st{0, 0, 0, 0, 0};
    // 1. openers with a local partner -> compact list (contiguous chunks)
    const uint32_t per = (tot + THREADS - 1) / THREADS;
    const uint32_t f0 = min(tot, tid * per), f1 = min(tot, f0 + per);
    uint32_t cnt = 0;
    uint32_t state = 0;
    int bl = f0 < f1 ? upper_index(T.off, nb, f0) : 0;
    for (uint32_t f = f0; f < f1; ++f) {
        while (f >= T.off[bl + 1])
            ++bl;
        const uint32_t r = rank0 + f;
        const uint32_t cs = T.cs[bl], ce = cs + T.n[bl];
        const uint32_t ic = r - cs;
        const bool opener = ((ic & 1u) == 0u) && (r + 1 < ce);
        if (opener && f + 1 < tot) {
            ++cnt;
        } else if (opener || (f == 0 && (ic & 1u))) {
            SeamRec rec;
            rec.s = get.s(f);
            rec.rank = r;
            rec.cell = a.bucket_cell[b0 + bl];
            rec.cs = cs;
            rec.n_c = T.n[bl];
            rec.step = step;
            if (opener) {
                a.seam_open[g] = rec;
                state |= 1u;
            } else {
                a.seam_close[g] = rec;
                state |= 2u;
            }
        }
    }
    if (state)
        atomicOr(&s_misc[2], state);
    uint32_t n_op;
    uint32_t w = block_exclusive_scan<THREADS>(cnt, red, &n_op);
    bl = f0 < f1 ? upper_index(T.off, nb, f0) : 0;
    for (uint32_t f = f0; f < f1 && cnt; ++f) {
        while (f >= T.off[bl + 1])
            ++bl;
        const uint32_t r = rank0 + f;
        const uint32_t cs = T.cs[bl], ce = cs + T.n[bl];
        const uint32_t ic = r - cs;
        if (((ic & 1u) == 0u) && (r + 1 < ce) && f + 1 < tot)
            opl[w++] = f;  // a full 32-bit position: groups here may exceed 2^16 records
    }
    __syncthreads();
    // 2. pairs, two consecutive openers per thread so that slots 2u, 2u+1
    //    share one Philox block when they are adjacent; an opener's bucket
    //    is found again from its position
    uint32_t shift = 0;
    if (n_op) {
        const uint32_t fa = opl[0];
        const int b = upper_index(T.off, nb, fa);
        shift = ((rank0 + fa - T.pc[b].slot_base) >> 1) & 1u;
    }
    for (uint32_t j = tid; 2 * j < n_op + shift; j += THREADS) {
        const int k0 = (int)(2 * j) - (int)shift;
        uint32_t qv[2] = {0, 0};
        double pv[2] = {0.0, 0.0};
        uint32_t runv[2] = {0, 0}, bv[2] = {0, 0};
        uint32_t sa[2] = {0, 0}, sb_[2] = {0, 0};
        uint64_t xa[2] = {0, 0}, xb[2] = {0, 0};
        bool valid[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int k = k0 + u;
            valid[u] = k >= 0 && k < (int)n_op;
            if (!valid[u])
                continue;
            const uint32_t f = opl[k];
            bv[u] = (uint32_t)upper_index(T.off, nb, f);
            const PairCtx &pc = T.pc[bv[u]];
            runv[u] = pc.run;
            qv[u] = (rank0 + f - pc.slot_base) >> 1;
            sa[u] = get.s(f);
            xa[u] = get.xi(f);
            const double va = get.v(f);
            sb_[u] = get.s(f + 1);
            xb[u] = get.xi(f + 1);
            const double vb = get.v(f + 1);
            pv[u] = pair_prob(a, pc, xa[u], va, xb[u], vb);
        }
        double phi[2] = {0.0, 0.0};
        if (valid[0] && valid[1] && (qv[0] & 1u) == 0u && qv[1] == qv[0] + 1 &&
            runv[0] == runv[1]) {
            const WordPair wp = philox_words(a.seed, runv[0], step, SDM_STREAM_GAMMA,
                                             qv[0] >> 1);
            phi[0] = word_to_uniform(wp.even);
            phi[1] = word_to_uniform(wp.odd);
        } else {
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (valid[u])
                    phi[u] = word_to_uniform(
                        philox_word(a.seed, runv[u], step, SDM_STREAM_GAMMA, qv[u]));
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (valid[u])
                finish_pair(a, T.pc[bv[u]], qv[u], pv[u], phi[u], sa[u], xa[u], sb_[u], xb[u],
                            st);
    }
    if (a.counters)
        store_group_stats<THREADS>(a, g, st, red);
    if (tid == 0) {
        a.seam_state[g] = s_misc[2];
        a.group_tot[g] = tot;
    }
}

struct GlobalGet {
    const uint32_t *ss;
    const uint64_t *xi_state;
    const double *v_state;
    __device__ uint32_t s(uint32_t f) const { return ss[f]; }
    __device__ uint64_t xi(uint32_t f) const { return xi_state ? xi_state[ss[f]] : 0; }
    __device__ double v(uint32_t f) const { return v_state ? v_state[ss[f]] : 0.0; }
};

__device__ __forceinline__ bool rec_less(uint32_t ba, uint64_t ka, uint32_t sa,
                                         uint32_t bb, uint64_t kb, uint32_t sbb)
{
    if (ba != bb)
        return ba < bb;
    if (ka != kb)
        return ka < kb;
    return sa < sbb;
}

// Shuffle key of SD s (fused mode): the same Philox word the tile kernel
// drew for it, element s - offset of its run.
__device__ __forceinline__ uint64_t shuffle_key(const GroupArgs &a, uint32_t s, uint32_t step)
{
    uint32_t run = a.run;
    uint64_t e = s;
    if (a.seg_off) {
        const int seg = find_seg(a.seg_off, a.n_cell, s);
        run = (uint32_t)a.seg_run[seg];
        e = (uint64_t)(s - a.seg_off[seg]);
    }
    return philox_word(a.seed, run, step, SDM_STREAM_SHUFFLE, e) >> 11;
}

// Local bucket of a record of this group.
__device__ __forceinline__ uint32_t local_bucket(const GroupArgs &a, int b0, int nb, uint64_t key,
                                                 uint32_t s)
{
    if (nb == 1)
        return 0;
    int c = 0;
    if (a.seg_off)
        c = find_seg(a.seg_off, a.n_cell, s);
    else if (a.cell_id)
        c = a.cell_id[s];
    const int h = a.cell_h[c];
    const uint32_t b = (uint32_t)a.cell_bucket_base[c] + (h ? (uint32_t)(key >> (53 - h)) : 0u);
    return b - (uint32_t)b0;
}

// The largest float not above x (x in [0, 1)).
__device__ __forceinline__ float float_below(double x)
{
    const float f = (float)x;
    return (double)f > x ? __uint_as_float(__float_as_uint(f) - 1u) : f;
}

// x >= 0 rounded up to single precision (NaN stays NaN, beyond the float
// range +inf), for testing a bound against phi held as float_below(phi)
__device__ __forceinline__ float float_above(double x)
{
    const float f = (float)x;
    return (double)f < x ? __uint_as_float(__float_as_uint(f) + 1u) : f;
}

// --------------------------------------------------------------- k_group
// The usual fused plans (seven records per thread, 39 KB of LDS) run three
// workgroups per CU: at most 80 VGPRs, six waves per SIMD.
template <int THREADS, int EPT, bool FUSED, bool ONE_CELL = false, bool WHOLE = false>
__global__ __launch_bounds__(THREADS, (FUSED && EPT <= 7) ? 6 : 4) void k_group(GroupArgs a)
{
    constexpr int CAP = THREADS * EPT;
    constexpr int NSUB = CAP;  // sub-buckets per group
    __shared__ uint32_t t_off[MAXB + 1];
    __shared__ uint32_t t_subbase[MAXB + 1];
    __shared__ uint32_t t_shift[MAXB];     // sub-bucket shift (whole key, or the 24 stored bits)
    __shared__ uint8_t t_cl[MAXB];         // the bucket's cell among the group's cells
    __shared__ uint32_t t_mask[MAXB];
    __shared__ uint32_t t_cs[MAXB];
    __shared__ uint32_t t_n[MAXB];
    __shared__ PairCtx t_pc[MAXB];
    __shared__ uint32_t t_pa[MAXB];        // first opener position of each bucket
    __shared__ uint32_t t_poff[MAXB + 1];  // pairs of the buckets before
    __shared__ uint8_t pair_bl[FUSED && !ONE_CELL ? CAP / 2 : 1];  // bucket of each pair
    // groups of whole cells: each pair's phi (rounded down) waits in LDS
    // rather than in registers through the sort
    __shared__ float phi_lds[FUSED && WHOLE ? CAP / 2 : 1];
    // direct starts: per-wave sums of the tiles' offsets of buckets b0 .. b1 - 1
    __shared__ uint32_t colpart[FUSED && (ONE_CELL || WHOLE) ? (THREADS / 64) * MAXB : 1];
    // cells of the group (c_lo + i): first bucket, key bits, run and, for
    // batches, first SD slot
    __shared__ uint32_t g_cbb[MAXB];
    __shared__ uint32_t g_ch[MAXB];
    __shared__ uint32_t g_run[MAXB];
    __shared__ uint32_t g_seg[MAXB + 1];
    // sub-bucket counts, then their exclusive sums (16 bits: at most CAP)
    __shared__ __align__(4) uint16_t sub_hist[NSUB + 2];
    uint32_t *sub_w = reinterpret_cast<uint32_t *>(sub_hist);
    __shared__ uint32_t red[5 * (THREADS / 64) + 8];  // scans and statistics
    __shared__ uint32_t s_misc[8];
    // gather: tile map and the group's run in every tile; sort: (key bits,
    // id) words (list modes: keys, then ids) by sub-bucket position;
    // afterwards the fused mode's bound codes in sorted order (their ids go
    // to the sub-bucket table, dead by then)
    constexpr int POOL = FUSED ? 8 * CAP : 12 * CAP;
    __shared__ __align__(16) unsigned char pool[POOL];
    static_assert(CAP < 65536, "16-bit sub-bucket sums and candidate positions");
    static_assert(2 * (NSUB + 2) >= 4 * (CAP / 2), "candidate list fits the sub-bucket table");
    static_assert(2 * CAP + 4 * (MAX_TILES + 1) + 4 * MAX_TILES <= POOL,
                  "run tables must fit the sort pool");
    // run_pre: the group's records before each tile's run; run_base: the
    // record slot of a group position li in tile t is run_base[t] + li
    uint32_t *run_pre = reinterpret_cast<uint32_t *>(pool + 2 * CAP);
    uint32_t *run_base = reinterpret_cast<uint32_t *>(pool + 2 * CAP + 4 * (MAX_TILES + 1));

    const int tid = threadIdx.x;
    const int g = xcd_local_index((int)blockIdx.x, (int)gridDim.x);
    const int b0 = a.group_first[g], b1 = a.group_first[g + 1];
    const int nb = b1 - b0;
    const int nt = a.n_tiles;
    const int64_t Bp = a.B + 1;
    constexpr bool fused = FUSED;
    // with dense tables, a single cell, or groups of whole cells, can take
    // their bucket starts from the tiles' own offsets: bucket b starts at
    // the sum over tiles of the tile's offset of b (known after the runs'
    // scan below)
    // (WHOLE: the instance for groups of whole cells)
    const bool direct = FUSED && (ONE_CELL || WHOLE) && a.direct;
    const bool directm = direct && WHOLE && !ONE_CELL;
    uint32_t rank0 = 0, tot = 0;
    if (!direct) {
        rank0 = a.bucket_start[b0];
        tot = a.bucket_start[b1] - rank0;
    }
    // (read here, so that the load overlaps the table loads below)
    const uint32_t step = step_of(a.step, a.step_dev);
    if (tid == 0) {
        s_misc[2] = 0;
        s_misc[3] = 0;  // listed candidate pairs (fused LDS path)
    }

    // (one cell: cell 0, no lookups)
    const int c_lo = ONE_CELL ? 0 : a.bucket_cell[b0];
    const int n_gc = ONE_CELL ? 1 : a.bucket_cell[b1 - 1] - c_lo + 1;  // <= nb <= MAXB
    // the tiles that can hold the group's records: all of them, except in a
    // batch, whose runs occupy contiguous slot ranges (tiles t_first ..
    // t_first + ntl - 1)
    int t_first = 0, ntl = nt;
    if (fused && a.seg_off) {
        const uint32_t s_lo = a.seg_off[c_lo], s_hi = a.seg_off[c_lo + n_gc];
        const uint32_t tile = (uint32_t)a.tile;
        t_first = s_hi > s_lo ? (int)(s_lo / tile) : 0;
        ntl = s_hi > s_lo ? min(nt - 1, (int)((s_hi - 1) / tile)) - t_first + 1 : 0;
    }

    // 1. this group's run in each of those tiles; bucket and cell tables.
    // With at most one run per thread the runs stay in registers until
    // their scan, whose barrier also completes the tables
    const bool runs_in_regs = ntl <= THREADS;
    uint32_t r_base = 0, r_cnt = 0;  // run t = tid (runs_in_regs)
    const bool dtv = tid < ntl;  // direct: this thread's tile and its offsets row
    const uint16_t *drow = a.tile_off + (int64_t)(dtv ? tid : 0) * Bp + b0;
    if (direct) {  // (ntl <= THREADS)
        const uint32_t lo = drow[0], hi = drow[nb];
        r_base = (uint32_t)tid * (uint32_t)a.tile + lo;
        r_cnt = dtv ? hi - lo : 0u;
        // rank0: the sum of the offsets of b0 (column 0)
        const uint32_t ws = wave_scan_u32(dtv ? lo : 0u);  // lane 63: the sum
        if ((tid & 63) == 63)
            colpart[(tid >> 6) * MAXB] = ws;
        if (directm) {  // every bucket's start: columns 1 .. nb - 1 too
            uint32_t v[MAXB];
#pragma unroll
            for (int j = 1; j < MAXB; ++j)
                v[j] = dtv ? (uint32_t)drow[min(j, nb)] : 0u;
#pragma unroll
            for (int j = 1; j < MAXB; ++j) {
                if (j < nb) {
                    const uint32_t wj = wave_scan_u32(v[j]);
                    if ((tid & 63) == 63)
                        colpart[(tid >> 6) * MAXB + j] = wj;
                }
            }
        }
    } else if (!a.tile_lb) {  // dense tables: both offsets load together
        for (int t = tid; t < ntl; t += THREADS) {
            const uint32_t lo = a.tile_offT[(int64_t)b0 * nt + t_first + t];
            const uint32_t hi = a.tile_offT[(int64_t)b1 * nt + t_first + t];
            r_base = (uint32_t)(t_first + t) * (uint32_t)a.tile + lo;
            r_cnt = hi - lo;
            if (!runs_in_regs) {
                run_base[t] = r_base;
                run_pre[t] = r_cnt;
            }
        }
    } else {  // local tables (tile_bucket_off for b0 and b1, branch-free)
        for (int t = tid; t < ntl; t += THREADS) {
            const int tt = t_first + t;
            const int lb = a.tile_lb[tt], tnb = a.tile_nb[tt];
            const uint32_t loff = a.tile_loff[tt];
            const int i0 = min(max(b0 - lb, 0), tnb), i1 = min(max(b1 - lb, 0), tnb);
            const uint32_t v0 = a.tile_off[loff + (uint32_t)i0];
            const uint32_t v1 = a.tile_off[loff + (uint32_t)i1];
            const uint32_t lo = b0 <= lb ? 0u : v0, hi = b1 <= lb ? 0u : v1;
            r_base = (uint32_t)tt * (uint32_t)a.tile + lo;
            r_cnt = hi - lo;
            if (!runs_in_regs) {
                run_base[t] = r_base;
                run_pre[t] = r_cnt;
            }
        }
    }
    // the bucket, cell and per-bucket tables start on other waves than the
    // runs (a thread index rotated by whole waves), so that their load
    // chains run side by side
    auto rot = [&](int k) { return (tid + (k % (THREADS / 64)) * 64) % THREADS; };
    for (int i = rot(4); i <= nb && !direct; i += THREADS)
        t_off[i] = a.bucket_start[b0 + i] - rank0;
    for (int i = rot(5); i <= n_gc; i += THREADS) {
        const int c = c_lo + i;
        if (i < n_gc) {
            g_cbb[i] = (uint32_t)a.cell_bucket_base[c];
            g_ch[i] = (uint32_t)a.cell_h[c];
            g_run[i] = a.seg_run ? (uint32_t)a.seg_run[c] : a.run;
        }
        if (a.seg_off)
            g_seg[i] = a.seg_off[c];
    }
    for (int i = rot(6); i < nb; i += THREADS) {
        const int b = b0 + i;
        const int c = ONE_CELL ? 0 : a.bucket_cell[b];
        const int h = a.cell_h[c];
        const int u = a.sub_bits[b];
        t_shift[i] = (uint32_t)(fused ? 24 - u : 53 - h - u);
        t_cl[i] = (uint8_t)(c - c_lo);
        t_mask[i] = (1u << u) - 1u;
        t_subbase[i] = 1u << u;
        int first = 0;
        uint32_t cs = 0, n_c;
        if (directm) {
            // the cell's buckets (inside the group) for now; its start, its
            // size and the pair constants that need them follow the scan
            first = a.cell_bucket_base[c];
            cs = (uint32_t)(first - b0);
            n_c = (uint32_t)(a.cell_bucket_base[c + 1] - b0);
        } else if (direct) {  // (one cell: buckets 0 .. B - 1, starting at rank 0)
            n_c = *a.n_total;
        } else {
            first = a.cell_bucket_base[c];
            const int last = a.cell_bucket_base[c + 1];
            cs = a.bucket_start[first];
            n_c = a.bucket_start[last] - cs;
        }
        t_cs[i] = cs;
        t_n[i] = n_c;
        // (directm: norm = dt / dV_c for now, F(2) = 1; times F(n_c) below)
        if (fused)
            t_pc[i] = directm ? pair_ctx(a, c, 0u, 2u) : pair_ctx(a, c, cs, n_c);
        if (b == first && !directm)
            a.cell_start[c] = cs;
    }
    // (the sub-bucket counts start at zero; the next barrier orders this)
    for (uint32_t i = tid; i < (uint32_t)(NSUB + 2) / 2; i += THREADS)
        sub_w[i] = 0;
    const uint32_t cap_here =
        a.group_cap >= 0 ? (uint32_t)min(a.group_cap, CAP) : (uint32_t)CAP;
    // tile of each gathered slot (LDS path): with many short runs, each
    // run's thread fills its own entries right after the scan
    uint16_t *tmap = reinterpret_cast<uint16_t *>(pool);
    bool lds_path = tot <= cap_here, own_fill = false;
    if (runs_in_regs) {
        uint32_t all;
        const uint32_t ex = block_exclusive_scan<THREADS>(r_cnt, red, &all);
        if (direct) {
            uint32_t r0 = 0;
#pragma unroll
            for (int w = 0; w < THREADS / 64; ++w)
                r0 += colpart[w * MAXB];
            rank0 = r0;
            tot = all;
            lds_path = tot <= cap_here;
            // the LDS path of one cell needs no bucket boundaries inside the
            // group (its pairs follow the ranks across them); the global path
            // sums the interior columns too
            if (!lds_path && !directm) {
                for (int i = 1; i < nb; ++i) {
                    const uint32_t ws = wave_scan_u32(dtv ? (uint32_t)drow[i] : 0u);
                    if ((tid & 63) == 63)
                        colpart[(tid >> 6) * MAXB + i] = ws;
                }
                __syncthreads();
            }
            if (tid <= nb) {
                uint32_t c = 0;
                if (tid > 0 && tid < nb && (!lds_path || directm)) {
#pragma unroll
                    for (int w = 0; w < THREADS / 64; ++w)
                        c += colpart[w * MAXB + tid];
                    c -= rank0;
                }
                t_off[tid] = tid == 0 ? 0u : tid == nb ? tot : c;
            }
        }
        own_fill = ntl > 8 && lds_path;
        if (tid < ntl) {
            run_pre[tid] = ex;
            run_base[tid] = r_base - ex;  // modulo 2^32; run_base[t] + li is the slot
            if (own_fill)
                for (uint32_t li = ex; li < ex + r_cnt; ++li)
                    tmap[li] = (uint16_t)tid;
        }
        if (tid == 0)
            run_pre[ntl] = all;
    } else {
        __syncthreads();
        lds_exclusive_scan<THREADS, (MAX_TILES + THREADS - 1) / THREADS>(run_pre, ntl, red);
        for (int t = tid; t < ntl; t += THREADS)
            run_base[t] -= run_pre[t];  // modulo 2^32; run_base[t] + li is the slot
    }
    if (tid < 64) {  // nb <= MAXB <= 64: one wave scans the sub-bucket counts
        // groups of whole cells (directm): each bucket's start (lane i: bucket
        // b0 + i, from rank0), then its cell's start and size, the pair
        // constants that need them and the cell's entry of cell_start
        uint32_t dm_lo = 0, dm_hi = 0, dm_cs = 0, dm_n = 0;
        if (directm) {
            uint32_t col = 0;
            if (tid > 0 && tid < nb) {
#pragma unroll
                for (int w = 0; w < THREADS / 64; ++w)
                    col += colpart[w * MAXB + tid];
                col -= rank0;
            } else if (tid == nb) {
                col = tot;
            }
            const int fi = tid < nb ? (int)t_cs[tid] : 0;  // the cell's first bucket
            const int la = tid < nb ? (int)t_n[tid] : 0;   // and one past its last
            const uint32_t cs_rel = (uint32_t)__shfl((int)col, fi);
            const uint32_t ce_rel = (uint32_t)__shfl((int)col, la);
            dm_hi = (uint32_t)__shfl((int)col, min(tid + 1, 63));
            dm_lo = col;
            dm_cs = rank0 + cs_rel;
            dm_n = ce_rel - cs_rel;
            if (tid < nb) {
                t_cs[tid] = dm_cs;
                t_n[tid] = dm_n;
                t_pc[tid].norm = t_pc[tid].norm * (double)pair_scale((uint64_t)dm_n);
                t_pc[tid].slot_base = a.slot_cell_local ? dm_cs : 0u;
                if (fi == tid)
                    a.cell_start[c_lo + (int)t_cl[tid]] = dm_cs;
            }
        }
        const uint32_t ns = tid < nb ? t_subbase[tid] : 0u;
        const uint32_t inc = wave_inclusive_scan(ns);
        if (tid < nb)
            t_subbase[tid] = inc - ns;
        if (tid == 63)
            t_subbase[nb] = inc;
        // pairs of every bucket, known before the sort: openers at even
        // in-cell indices whose closer is in the same cell and in this
        // group; pair k of the group opens at t_pa[b] + 2 (k - t_poff[b])
        uint32_t cnt = 0;
        if (direct && ONE_CELL) {
            // one cell, its ranks rank0 .. rank0 + tot - 1 as one range (the
            // openers of every bucket, counted together)
            if (tid == 0) {
                const uint32_t fa = rank0 & 1u;  // (the cell starts at rank 0)
                if (tot > 0) {
                    const uint32_t lim = min(tot - 1u, t_n[0] - 1u - rank0);
                    cnt = fa < lim ? (lim - fa + 1u) >> 1 : 0u;
                }
                t_pa[0] = fa;
            }
        } else if (tid < nb) {
            const uint32_t lo = directm ? dm_lo : t_off[tid];
            const uint32_t hi = directm ? dm_hi : t_off[tid + 1];
            const uint32_t cs = directm ? dm_cs : t_cs[tid];
            const uint32_t n_c = directm ? dm_n : t_n[tid];
            const uint32_t fa = lo + ((rank0 + lo - cs) & 1u);
            if (lo < hi) {
                // openers f < lim: f < hi, f + 1 < tot, rank0 + f + 1 < cs + n_c
                uint32_t lim = min(hi, tot - 1u);
                lim = min(lim, cs + n_c - 1u - rank0);
                cnt = fa < lim ? (lim - fa + 1u) >> 1 : 0u;
            }
            t_pa[tid] = fa;
        }
        const uint32_t pinc = wave_inclusive_scan(cnt);
        if (tid < nb)
            t_poff[tid] = pinc - cnt;
        if (tid == 63)
            t_poff[nb] = pinc;
    }
    __syncthreads();

    if (lds_path) {
        // 2. gather the records (every thread keeps its EPT records in
        //    registers), counting sort by (bucket, next key bits) in LDS,
        //    then each thread ranks its own records by (key, s) within
        //    their sub-bucket
        uint64_t *K1 = reinterpret_cast<uint64_t *>(pool);
        uint32_t *S1 = reinterpret_cast<uint32_t *>(pool + 8 * CAP);
        const uint32_t nsub = t_subbase[nb];
        if (!own_fill) {
            if (ntl <= 8) {  // a few long runs (batches): every thread on each
                for (int t = 0; t < ntl; ++t)
                    for (uint32_t li = run_pre[t] + tid; li < run_pre[t + 1]; li += THREADS)
                        tmap[li] = (uint16_t)t;
            } else {         // many short runs: a thread per run
                for (int t = tid; t < ntl; t += THREADS)
                    for (uint32_t li = run_pre[t]; li < run_pre[t + 1]; ++li)
                        tmap[li] = (uint16_t)t;
            }
            __syncthreads();
        }
        // fused mode: the record carries the 24 key bits below its bucket's
        // (bits 28 - h .. 52 - h) and the bucket's low 8 bits; they fix the
        // bucket and sub-bucket (u <= 24), and the rank falls back to the
        // whole key only between equal stored bits
        uint64_t key[EPT];
        uint32_t cod[EPT];  // fused mode: the bound codes
        uint32_t sid[EPT], sbk[EPT], fp[EPT];
        uint8_t blk[EPT], gcl[EPT];
        // every thread loads all its slots unconditionally (slots past tot
        // repeat the last record and are dropped below), so that the loads
        // of all EPT records are in flight together
        const uint32_t last = tot > 0 ? tot - 1 : 0;
        // fused mode: phi of this thread's pairs (k = 2j, 2j + 1, j = tid +
        // it THREADS), drawn while the records are in flight
        constexpr int PITER = (CAP / 2 + 2 * THREADS - 1) / (2 * THREADS);
        const uint32_t n_pairs = t_poff[nb];
        // openers every second position (ONE_CELL: a single-cell launch)
        const bool one_cell = ONE_CELL || n_gc == 1;
        // kept as floats rounded down (phi_lo <= phi), so that the bound test
        // below stays conservative; listed pairs draw phi again exactly
        float phi_pre[PITER][2];
        if (tot > 0 && fused) {
            uint64_t rr[EPT];
            int tt[EPT];
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t li = min((uint32_t)(e * THREADS + tid), last);
                tt[e] = tmap[li];
                rr[e] = a.rec_f[run_base[tt[e]] + li];
            }
#pragma unroll
            for (int it = 0; it < PITER; ++it) {
                const uint32_t j = (uint32_t)tid + (uint32_t)it * THREADS;
                uint32_t qv[2] = {0, 0}, runv[2] = {0, 0};
                bool valid[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const uint32_t k = 2 * j + (uint32_t)u;
                    valid[u] = k < n_pairs;
                    phi_pre[it][u] = 0.0f;
                    if (!valid[u])
                        continue;
                    int bl = 0;
                    uint32_t f = t_pa[0] + 2u * k;
                    if (!one_cell) {
                        bl = upper_index(t_poff, nb, k);
                        f = t_pa[bl] + 2u * (k - t_poff[bl]);
                    }
                    if (!one_cell)
                        pair_bl[k] = (uint8_t)bl;
                    runv[u] = t_pc[bl].run;
                    qv[u] = (rank0 + f - t_pc[bl].slot_base) >> 1;
                }
                if (valid[1] && (qv[0] & 1u) == 0u && qv[1] == qv[0] + 1u &&
                    runv[0] == runv[1]) {
                    const WordPair wp = philox_words(a.seed, runv[0], step, SDM_STREAM_GAMMA,
                                                     qv[0] >> 1);
                    phi_pre[it][0] = float_below(word_to_uniform(wp.even));
                    phi_pre[it][1] = float_below(word_to_uniform(wp.odd));
                } else {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        if (valid[u])
                            phi_pre[it][u] = float_below(word_to_uniform(
                                philox_word(a.seed, runv[u], step, SDM_STREAM_GAMMA, qv[u])));
                }
                if (WHOLE) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        if (valid[u])
                            phi_lds[2 * j + (uint32_t)u] = phi_pre[it][u];
                }
            }
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint64_t r = rr[e];
                sid[e] = (uint32_t)(t_first + tt[e]) * (uint32_t)a.tile +
                         ((uint32_t)r & ((1u << RF_BKT_SHIFT) - 1u));
                key[e] = (r >> RF_BKT_SHIFT) & ((1ull << (RF_XC_SHIFT - RF_BKT_SHIFT)) - 1ull);
                cod[e] = (uint32_t)(r >> RF_XC_SHIFT);
            }
        } else if (tot > 0) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t li = min((uint32_t)(e * THREADS + tid), last);
                const int t = tmap[li];
                const uint32_t pos = run_base[t] + li;
                const RecK rk = a.rec_k[pos];
                key[e] = rk.key;
                sid[e] = rk.s;
                cod[e] = 0;
            }
        }
        if (fused && tot == 0) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                sbk[e] = 0xFFFFFFFFu;
                blk[e] = 0;
                gcl[e] = 0;
                fp[e] = 0;
            }
        } else if (fused) {
            // the bucket from its low 5 bits (a group spans <= 32 buckets);
            // key[] keeps the 24 key bits.  Branch-free over the EPT records
            // (slots past tot hold the last record and count nothing), so
            // that the table reads, then the counting atomics, are in
            // flight together
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const bool ok = (uint32_t)(e * THREADS + tid) < tot;
                const uint32_t bl = ((uint32_t)key[e] - (uint32_t)b0) & 31u;
                key[e] = (key[e] >> (RF_KEY_SHIFT - RF_BKT_SHIFT)) & 0xFFFFFFu;
                const uint32_t sub = (uint32_t)(key[e] >> t_shift[bl]) & t_mask[bl];
                gcl[e] = ok && !ONE_CELL ? t_cl[bl] : (uint8_t)0;  // (one cell: cell 0)
                blk[e] = ok ? (uint8_t)bl : (uint8_t)0;
                sbk[e] = ok ? t_subbase[bl] + sub : 0xFFFFFFFFu;
                // rank among equal sub-buckets: a 16-bit count in half of
                // an LDS word (it never carries into the other half)
                const uint32_t sh = (sbk[e] & 1u) * 16u;
                // (a slot past tot adds 0 to a word of its own lane)
                const uint32_t old =
                    atomicAdd(&sub_w[ok ? sbk[e] >> 1 : (uint32_t)(tid & 63)], ok ? 1u << sh : 0u);
                fp[e] = ok ? (old >> sh) & 0xFFFFu : 0u;
            }
        }
        if (!fused) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t li = (uint32_t)(e * THREADS + tid);
                sbk[e] = 0xFFFFFFFFu;
                blk[e] = 0;
                gcl[e] = 0;
                fp[e] = 0;
                if (li < tot) {
                    // the record's cell among the group's cells
                    int cl = 0;
                    if (a.seg_off)
                        cl = upper_index(g_seg, n_gc, sid[e]);
                    else if (a.cell_id && n_gc > 1)
                        cl = a.cell_id[sid[e]] - c_lo;
                    gcl[e] = (uint8_t)cl;
                    const uint32_t h = g_ch[cl];
                    const uint32_t bl =
                        g_cbb[cl] - (uint32_t)b0 + (h ? (uint32_t)(key[e] >> (53 - h)) : 0u);
                    const uint32_t sub = (uint32_t)(key[e] >> t_shift[bl]) & t_mask[bl];
                    blk[e] = (uint8_t)bl;
                    sbk[e] = t_subbase[bl] + sub;
                    const uint32_t sh = (sbk[e] & 1u) * 16u;
                    fp[e] = (atomicAdd(&sub_w[sbk[e] >> 1], 1u << sh) >> sh) & 0xFFFFu;
                }
            }
        }
        __syncthreads();
        lds_exclusive_scan16<THREADS, (NSUB + THREADS - 1) / THREADS>(sub_hist, (int)nsub, red);
        // rank by (key, s) inside the sub-bucket: the first RW entries of
        // every sub-bucket with independent (predicated) loads, the rare
        // longer ones in a loop.  Fused mode sorts (24 stored key bits, id)
        // words and settles equal stored bits by the whole keys.
        constexpr uint32_t RW = 4;
        uint32_t rlo[EPT], rhi[EPT];
        uint32_t tie = 0;  // bit e: record e met an equal key (other id)
        if (fused) {
            uint64_t *KS = reinterpret_cast<uint64_t *>(pool);
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                if (sbk[e] != 0xFFFFFFFFu)
                    KS[sub_hist[sbk[e]] + fp[e]] = (key[e] << 32) | sid[e];
            __syncthreads();
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const bool ok = sbk[e] != 0xFFFFFFFFu;
                const uint32_t sb = ok ? sbk[e] : 0u;
                const uint32_t lo = sub_hist[sb], hi = sub_hist[sb + 1];
                rlo[e] = lo;
                rhi[e] = ok ? hi : lo;
            }
            // the window compares only the key-bit words (the high word of
            // each entry); a record meets its own entry once, so two or more
            // equal words mean another record with the same stored bits
            const uint32_t *KW = reinterpret_cast<const uint32_t *>(pool) + 1;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t hm = (uint32_t)key[e];
                uint32_t hq[RW];
#pragma unroll
                for (uint32_t j = 0; j < RW; ++j)
                    hq[j] = KW[2u * min(rlo[e] + j, (uint32_t)CAP - 1u)];
                uint32_t r = 0, eq = 0;
#pragma unroll
                for (uint32_t j = 0; j < RW; ++j) {
                    const bool in = rlo[e] + j < rhi[e];
                    r += in && hq[j] < hm;
                    eq += in && hq[j] == hm;
                }
                for (uint32_t q = rlo[e] + RW; q < rhi[e]; ++q) {
                    const uint32_t h = KW[2u * q];
                    r += h < hm;
                    eq += h == hm;
                }
                if (eq > 1)
                    tie |= 1u << e;
                fp[e] = rlo[e] + r;
            }
            if (tie) {
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    if (!((tie >> e) & 1u))
                        continue;
                    // equal stored bits: the whole keys (same cell, so the same
                    // run) decide, then the ids
                    const int cl = gcl[e];
                    const uint32_t so = a.seg_off ? g_seg[cl] : 0u;
                    const uint32_t run = g_run[cl];
                    const uint32_t hm = (uint32_t)key[e];
                    const uint64_t km =
                        philox_word(a.seed, run, step, SDM_STREAM_SHUFFLE, sid[e] - so) >> 11;
                    for (uint32_t q = rlo[e]; q < rhi[e]; ++q) {
                        const uint64_t w = KS[q];
                        const uint32_t sq = (uint32_t)w;
                        if ((uint32_t)(w >> 32) != hm || sq == sid[e])
                            continue;
                        const uint64_t kx =
                            philox_word(a.seed, run, step, SDM_STREAM_SHUFFLE, sq - so) >> 11;
                        fp[e] += (kx < km) || (kx == km && sq < sid[e]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                if (sbk[e] != 0xFFFFFFFFu) {
                    const uint32_t pos = sub_hist[sbk[e]] + fp[e];
                    K1[pos] = key[e];
                    S1[pos] = sid[e];
                }
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const uint32_t sb = sbk[e] != 0xFFFFFFFFu ? sbk[e] : 0u;
                rlo[e] = sub_hist[sb];
                rhi[e] = sbk[e] != 0xFFFFFFFFu ? sub_hist[sb + 1] : rlo[e];
            }
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                uint32_t r = 0;
                for (uint32_t q = rlo[e]; q < rhi[e]; ++q) {
                    const uint64_t kq = K1[q];
                    r += (kq < key[e]) || (kq == key[e] && S1[q] < sid[e]);
                }
                fp[e] = rlo[e] + r;
            }
        }
        __syncthreads();  // keys and ids are dead
        if (!fused) {
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                if (sbk[e] != 0xFFFFFFFFu)
                    a.idx_out[rank0 + fp[e]] = sid[e];
            return;
        }

        // 3. ids and bound codes in sorted order, idx, seams
        uint32_t *RC = reinterpret_cast<uint32_t *>(pool);
        uint32_t *RS = reinterpret_cast<uint32_t *>(pool + 4 * CAP);
        // position -> slot: the low two bits XORed with bits 4-5, so that
        // lanes reading positions 4 apart (two pairs per thread) hit
        // different LDS banks; a permutation within every 4 positions
        auto sw = [](uint32_t f) { return f ^ ((f >> 4) & 3u); };
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if (sbk[e] == 0xFFFFFFFFu)
                continue;
            const uint32_t f = fp[e];
            RC[sw(f)] = cod[e];
            RS[sw(f)] = sid[e];
        }
        __syncthreads();
        for (uint32_t f = tid; f < tot; f += THREADS)
            a.idx_out[rank0 + f] = RS[sw(f)];
        if (tid == 0 && tot > 0) {
            // a closer at position 0 and an opener at position tot - 1 pair
            // with the neighbouring groups (k_finish)
            uint32_t state = 0;
            for (int end = 0; end < 2; ++end) {
                const uint32_t f = end ? tot - 1u : 0u;
                const int bl = ONE_CELL ? 0 : upper_index(t_off, nb, f);
                const uint32_t cs = t_cs[bl];
                const uint32_t ic = rank0 + f - cs;
                const bool seam = end ? ((ic & 1u) == 0u && ic + 1u < t_n[bl]) : (ic & 1u) != 0u;
                if (!seam)
                    continue;
                SeamRec rec;
                rec.s = RS[sw(f)];
                rec.rank = rank0 + f;
                rec.cell = c_lo + (int)t_cl[bl];
                rec.cs = cs;
                rec.n_c = t_n[bl];
                rec.step = step;
                if (end) {
                    a.seam_open[g] = rec;
                    state |= 1u;
                } else {
                    a.seam_close[g] = rec;
                    state |= 2u;
                }
            }
            a.seam_state[g] = state;
            a.group_tot[g] = tot;
        }
        if (tid == 0 && tot == 0) {
            a.seam_state[g] = 0;
            a.group_tot[g] = 0;
        }

        // 4. pairs k = 2j, 2j + 1 per thread (phi drawn during the gather):
        //    the bound of eq. (3) from the codes against phi.
        //    Pairs it does not rule out go to a list (position | bucket <<
        //    16, in the dead sub-bucket table); after a barrier one thread
        //    per listed pair reads xi and the attributes from the state
        //    (one round trip for the group) for the exact eq. (3), gamma
        //    and eqs. (4)-(6)
        Stats st{0, 0, 0, 0, 0};
        uint32_t *CL = sub_w;  // the sub-bucket table is dead after the ranks
#pragma unroll
        for (int it = 0; it < PITER; ++it) {
            const uint32_t j = (uint32_t)tid + (uint32_t)it * THREADS;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const uint32_t k = 2 * j + (uint32_t)u;
                if (k >= n_pairs)
                    continue;
                int bl = 0;
                uint32_t f = t_pa[0] + 2u * k;
                if (!one_cell) {
                    bl = pair_bl[k];
                    f = t_pa[bl] + 2u * (k - t_poff[bl]);
                }
                const PairCtx &pc = t_pc[bl];
                const double pub = pair_bound(pc, RC[sw(f)], RC[sw(f + 1)]);
                // (several cells: the test in single precision, pub rounded
                // up, so that no doubles of phi wait in registers)
                const bool below = ONE_CELL ? pub < (double)phi_pre[it][u]
                                            : float_above(pub) < (WHOLE ? phi_lds[k] : phi_pre[it][u]);
                if (below) {  // gamma = -0.0: no collision
                    st.pairs += 1;
                    if (a.gamma_out)
                        a.gamma_out[pc.gbase + ((rank0 + f - pc.slot_base) >> 1)] = -0.0;
                } else {
                    CL[atomicAdd(&s_misc[3], 1u)] = f | ((uint32_t)bl << 16);
                }
            }
        }
        __syncthreads();
        const uint32_t n_cand = s_misc[3];
        for (uint32_t i = tid; i < n_cand; i += THREADS) {
            const uint32_t f = CL[i] & 0xFFFFu;
            const PairCtx &pc = t_pc[CL[i] >> 16];
            const uint32_t q = (rank0 + f - pc.slot_base) >> 1;
            const uint32_t sa = RS[sw(f)], sb2 = RS[sw(f + 1)];
            const uint64_t xa = a.xi[sa], xb = a.xi[sb2];
            const double va = a.attr[sa], vb = a.attr[sb2];
            const double phi =
                word_to_uniform(philox_word(a.seed, pc.run, step, SDM_STREAM_GAMMA, q));
            const double p = pair_prob(a, pc, xa, va, xb, vb);
            finish_pair_v(a, pc, q, p, phi, sa, xa, va, sb2, xb, vb, st);
        }
        if (a.counters)
            store_group_stats<THREADS>(a, g, st, red);
        return;
    }
    const GroupTabs T{t_off, t_cs, t_n, t_pc};

    // ---------------------------------------------------- global path
    // The group's records are gathered into scratch at [2 rank0, 2 rank0 + P),
    // P = next power of two >= tot (ranges of consecutive groups are disjoint
    // since P <= 2 tot), and sorted there by (bucket, key, s) with a bitonic
    // network.  The pair phase then reads xi and v from the state; its
    // opener list reuses the group's bucket scratch.
    const uint32_t base2 = 2u * rank0;
    uint32_t P = 1;
    while (P < tot)
        P <<= 1;
    for (uint32_t li = tid; li < tot; li += THREADS) {
        const int t = upper_index(run_pre, ntl, li);
        const uint32_t pos = run_base[t] + li;
        const uint32_t s =
            fused ? (uint32_t)(t_first + t) * (uint32_t)a.tile +
                        ((uint32_t)a.rec_f[pos] & ((1u << RF_BKT_SHIFT) - 1u))
                  : a.rec_k[pos].s;
        const uint64_t k =
            fused ? shuffle_key(a, s, step) : a.rec_k[pos].key;
        a.sk[base2 + li] = k;
        a.ss[base2 + li] = s;
        a.sb[base2 + li] = local_bucket(a, b0, nb, k, s);
    }
    for (uint32_t i = tot + tid; i < P; i += THREADS) {
        a.sk[base2 + i] = ~0ull;
        a.ss[base2 + i] = ~0u;
        a.sb[base2 + i] = ~0u;
    }
    __threadfence_block();
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < P; i += THREADS) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint32_t bi = a.sb[base2 + i], bl2 = a.sb[base2 + l];
                    const uint64_t ki = a.sk[base2 + i], kl = a.sk[base2 + l];
                    const uint32_t si = a.ss[base2 + i], sl = a.ss[base2 + l];
                    const bool up = (i & k) == 0;
                    const bool gt = rec_less(bl2, kl, sl, bi, ki, si);
                    if (up ? gt : !gt) {
                        a.sb[base2 + i] = bl2;
                        a.sb[base2 + l] = bi;
                        a.sk[base2 + i] = kl;
                        a.sk[base2 + l] = ki;
                        a.ss[base2 + i] = sl;
                        a.ss[base2 + l] = si;
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
    }
    GlobalGet get{a.ss + base2, fused ? a.xi : nullptr, fused ? a.attr : nullptr};
    group_outputs<THREADS>(a, g, b0, nb, tot, rank0, T, get, red, s_misc, a.sb + base2);
}

// -------------------------------------------------------------- k_finish
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_finish(FinishArgs a)
{
    __shared__ uint32_t red[5 * (THREADS / 64) + 8];
    const int g = blockIdx.x * THREADS + threadIdx.x;
    Stats st{0, 0, 0, 0, 0};
    const bool fused = a.mode == MODE_FUSED;
    // the live total, loaded at once (its use is the block's last step)
    const bool keeper = blockIdx.x == 0 && threadIdx.x == 0;
    const uint32_t n_live = keeper ? a.n_acc[0] : 0u;
    if (fused && g < a.G) {
        // the next group's records are read before knowing they are needed
        // (one dependent round trip instead of three)
        const uint32_t state = a.seam_state[g];
        SeamRec op = a.seam_open[g];
        int g2 = g + 1;
        SeamRec cl;
        uint32_t tot2 = 0;
        if (g2 < a.G) {
            cl = a.seam_close[g2];
            tot2 = a.group_tot[g2];
        }
        if (a.counters) {
            const uint32_t *gs = a.group_stats + (int64_t)g * 5;
            st.pairs = gs[0];
            st.coll = gs[1];
            st.capped = gs[2];
            st.zeroed = gs[3];
            st.ge2 = gs[4];
        }
        if (state & 1u) {
            if (g2 < a.G && tot2 == 0) {
                while (g2 < a.G && a.group_tot[g2] == 0)
                    ++g2;
                if (g2 < a.G)
                    cl = a.seam_close[g2];
            }
            if (g2 < a.G) {
                // the step the group kernel drew its numbers for travels in
                // the record, so that no block reads the step counter that
                // block 0 advances
                const uint32_t step = op.step;
                const PairCtx pc = pair_ctx(a, op.cell, op.cs, op.n_c);
                const uint32_t q = (op.rank - pc.slot_base) >> 1;
                const uint64_t xo = a.xi[op.s], xc = a.xi[cl.s];
                const double vo = a.attr[op.s], vc = a.attr[cl.s];
                const double p = pair_prob(a, pc, xo, vo, xc, vc);
                const double phi =
                    word_to_uniform(philox_word(a.seed, pc.run, step, SDM_STREAM_GAMMA, q));
                finish_pair_v(a, pc, q, p, phi, op.s, xo, vo, cl.s, xc, vc, st);
            }
        }
    }
    if (fused && a.counters)
        flush_stats<THREADS>(st, a.counters, red);
    if (keeper) {
        const uint32_t n = n_live;
        *a.n_live_out = (int64_t)n;
        a.cell_start[a.n_cell] = n;
        a.n_acc[0] = 0;
        if (a.step_advance)
            *a.step_advance = *a.step_advance + 1u;
    }
}

// --------------------------------------------------------------- k_small
// A whole single-cell timestep in one workgroup, for launches of at most
// SMALL_CAP SD slots (the validation box of Sec. 4 has 2^13): the Philox
// keys, the sort by (key, s) in LDS (counting sort by the top 13 key bits,
// then each record's exact rank within its sub-bucket by whole keys), the
// pairs with gamma and eqs. (4)-(6), idx and the bookkeeping -- one launch
// per step where the general path takes four, each at its launch-latency
// floor at this size.  Results equal the general path's bit for bit.
constexpr int SMALL_THREADS = 1024;
constexpr int SMALL_EPT = 8;
constexpr int SMALL_CAP = SMALL_THREADS * SMALL_EPT;
constexpr int SMALL_SUB_SHIFT = 53 - 13;  // 2^13 = SMALL_CAP sub-buckets

struct SmallArgs {
    int64_t n_sd;
    uint64_t *xi;
    double *attr;
    int32_t n_attr;
    int64_t stride;
    uint64_t seed;
    uint32_t run;
    uint32_t step;
    const uint32_t *step_dev;
    uint32_t *step_advance;
    double dt;
    const double *dv_cell;
    double dv;
    KernelDesc kern;
    int slot_cell_local;
    uint32_t *idx_out;
    uint32_t *cell_start;
    int64_t *n_live_out;
    uint64_t *counters;
    double *gamma_out;
    // a single run: no segment tables (the pair helpers test seg_run)
    const uint32_t *seg_off;
    const int32_t *seg_run;
    const int32_t *seg_kernel;
    const double *seg_dv;
    const KernelDesc *kernels;
};

__global__ __launch_bounds__(SMALL_THREADS) void k_small(SmallArgs a)
{
    __shared__ uint64_t K[SMALL_CAP];                 // keys, by sub-bucket
    __shared__ uint16_t S[SMALL_CAP];                 // their slots
    __shared__ __align__(4) uint16_t H[SMALL_CAP + 2];  // sub-bucket counts, then starts
    __shared__ uint16_t R[SMALL_CAP];                 // slot of every rank
    __shared__ uint32_t red[5 * (SMALL_THREADS / 64) + 8];
    uint32_t *Hw = reinterpret_cast<uint32_t *>(H);
    const int tid = threadIdx.x;
    const int64_t n_items = a.n_sd;
    const uint32_t step = step_of(a.step, a.step_dev);
    for (int i = tid; i < (SMALL_CAP + 2) / 2; i += SMALL_THREADS)
        Hw[i] = 0;
    // 1. keys of the live slots (two slots per Philox block), all loads of
    //    xi in flight together
    uint64_t key[SMALL_EPT];
    uint32_t sb[SMALL_EPT], fp[SMALL_EPT];
    ulonglong2 xx[SMALL_EPT / 2];
#pragma unroll
    for (int k = 0; k < SMALL_EPT / 2; ++k) {
        const int64_t i0 = 2 * ((int64_t)k * SMALL_THREADS + tid);
        xx[k] = i0 + 1 < n_items ? *reinterpret_cast<const ulonglong2 *>(a.xi + i0)
                                 : make_ulonglong2(i0 < n_items ? a.xi[i0] : 0ull, 0ull);
    }
    __syncthreads();  // H cleared
    uint32_t live_n = 0;
#pragma unroll
    for (int k = 0; k < SMALL_EPT / 2; ++k) {
        const uint64_t p = (uint64_t)k * SMALL_THREADS + tid;
        const WordPair w = philox_words(a.seed, a.run, step, SDM_STREAM_SHUFFLE, p);
        const uint64_t kk[2] = {w.even >> 11, w.odd >> 11};
        const uint64_t xv[2] = {xx[k].x, xx[k].y};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int j = 2 * k + e;
            key[j] = kk[e];
            sb[j] = 0xFFFFFFFFu;
            fp[j] = 0;
            if (xv[e] > 0 && (int64_t)(2 * p + e) < n_items) {
                sb[j] = (uint32_t)(kk[e] >> SMALL_SUB_SHIFT);
                const uint32_t sh = (sb[j] & 1u) * 16u;
                fp[j] = (atomicAdd(&Hw[sb[j] >> 1], 1u << sh) >> sh) & 0xFFFFu;
                ++live_n;
            }
        }
    }
    uint32_t n;
    (void)block_exclusive_scan<SMALL_THREADS>(live_n, red, &n);
    __syncthreads();
    // 2. sub-bucket starts; records in sub-bucket order
    lds_exclusive_scan16<SMALL_THREADS, SMALL_EPT>(H, SMALL_CAP, red);
#pragma unroll
    for (int j = 0; j < SMALL_EPT; ++j) {
        if (sb[j] != 0xFFFFFFFFu) {
            const uint32_t q = H[sb[j]] + fp[j];
            K[q] = key[j];
            S[q] = (uint16_t)(2 * ((j >> 1) * SMALL_THREADS + tid) + (j & 1));
        }
    }
    __syncthreads();
    // 3. exact ranks by (key, s) within the sub-bucket: the first RW entries
    //    of every record's sub-bucket with independent loads (a sub-bucket
    //    holds one record on average), the rare longer ones in a loop
    constexpr uint32_t RW = 3;
    uint32_t lo[SMALL_EPT], hi[SMALL_EPT];
#pragma unroll
    for (int j = 0; j < SMALL_EPT; ++j) {
        const uint32_t b = sb[j] != 0xFFFFFFFFu ? sb[j] : 0u;
        lo[j] = H[b];
        hi[j] = sb[j] != 0xFFFFFFFFu ? H[b + 1] : lo[j];
    }
#pragma unroll
    for (int j = 0; j < SMALL_EPT; ++j) {
        const uint32_t s = 2u * ((uint32_t)(j >> 1) * SMALL_THREADS + (uint32_t)tid) + (uint32_t)(j & 1);
        uint32_t r = lo[j];
        uint64_t kq[RW];
        uint32_t sq[RW];
#pragma unroll
        for (uint32_t i = 0; i < RW; ++i) {  // loads first, no branches
            const uint32_t q = min(lo[j] + i, (uint32_t)SMALL_CAP - 1u);
            kq[i] = K[q];
            sq[i] = S[q];
        }
#pragma unroll
        for (uint32_t i = 0; i < RW; ++i) {
            const uint32_t lt = (uint32_t)(kq[i] < key[j]) |
                                ((uint32_t)(kq[i] == key[j]) & (uint32_t)(sq[i] < s));
            r += (lo[j] + i < hi[j]) ? lt : 0u;
        }
        for (uint32_t q = lo[j] + RW; q < hi[j]; ++q) {
            const uint64_t kq = K[q];
            r += (kq < key[j]) || (kq == key[j] && (uint32_t)S[q] < s);
        }
        if (sb[j] != 0xFFFFFFFFu)
            R[r] = (uint16_t)s;
    }
    __syncthreads();
    // 4. idx and the cell bookkeeping
    for (uint32_t i = tid; i < n; i += SMALL_THREADS)
        a.idx_out[i] = R[i];
    if (tid == 0) {
        *a.n_live_out = (int64_t)n;
        a.cell_start[0] = 0;
        a.cell_start[1] = n;
    }
    // 5. pairs (2q, 2q + 1) of the sorted cell, two per thread sharing a
    //    Philox block for phi
    const PairCtx pc = pair_ctx(a, 0, 0u, n);
    const uint32_t n_pairs = n / 2;
    Stats st{0, 0, 0, 0, 0};
    //    every pair's state loads issued before the first is used (the
    //    pairs of a thread: q = 2 jb + u, jb = tid, tid + THREADS)
    constexpr int PJ = SMALL_CAP / 4 / SMALL_THREADS;  // Philox blocks per thread
    uint32_t ps[PJ][2][2];
    uint64_t px[PJ][2][2];
    double pv[PJ][2][2];
#pragma unroll
    for (int i = 0; i < PJ; ++i)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            // pairs past the last read slot 0 (always a slot of the launch)
            const uint32_t q = 2 * ((uint32_t)tid + (uint32_t)i * SMALL_THREADS) + (uint32_t)u;
            ps[i][u][0] = q < n_pairs ? (uint32_t)R[2 * q] : 0u;
            ps[i][u][1] = q < n_pairs ? (uint32_t)R[2 * q + 1] : 0u;
        }
#pragma unroll
    for (int i = 0; i < PJ; ++i)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                px[i][u][e] = a.xi[ps[i][u][e]];
                pv[i][u][e] = a.attr[ps[i][u][e]];
            }
#pragma unroll
    for (int i = 0; i < PJ; ++i) {
        const uint32_t jb = (uint32_t)tid + (uint32_t)i * SMALL_THREADS;
        if (2 * jb >= n_pairs)
            continue;
        const WordPair wp = philox_words(a.seed, a.run, step, SDM_STREAM_GAMMA, jb);
        const double phi[2] = {word_to_uniform(wp.even), word_to_uniform(wp.odd)};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint32_t q = 2 * jb + (uint32_t)u;
            if (q >= n_pairs)
                continue;
            const double p = pair_prob(a, pc, px[i][u][0], pv[i][u][0], px[i][u][1], pv[i][u][1]);
            finish_pair_v(a, pc, q, p, phi[u], ps[i][u][0], px[i][u][0], pv[i][u][0],
                          ps[i][u][1], px[i][u][1], pv[i][u][1], st);
        }
    }
    flush_stats<SMALL_THREADS>(st, a.counters, red);
    if (tid == 0 && a.step_advance)
        *a.step_advance = *a.step_advance + 1u;
}

// =================================================================== host
static void *dalloc(Plan *p, size_t bytes)
{
    void *ptr = nullptr;
    if (bytes == 0)
        bytes = 8;
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess)
        throw HipError{e, "hipMalloc(plan workspace)"};
    p->allocs.push_back(ptr);
    return ptr;
}

template <class T>
static T *upload(Plan *p, const std::vector<T> &v)
{
    T *d = (T *)dalloc(p, sizeof(T) * std::max<size_t>(v.size(), 1));
    if (!v.empty())
        SDM_HIP(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return d;
}

void free_plan(Plan *p)
{
    if (!p)
        return;
    for (void *ptr : p->allocs)
        (void)hipFree(ptr);
    delete p;
}

static int ceil_log2_u64(uint64_t x)
{
    int b = 0;
    while ((1ull << b) < x)
        ++b;
    return b;
}

// Tile kernel LDS: the bucket histogram plus a staging buffer of at least
// 1024 records (the records of a tile leave in passes of `chunk`).
static int tile_hist_bytes(int B)
{
    return ((B + 1) * 4 + 15) & ~15;
}

static uint32_t tile_chunk_for(int B, int tile)
{
    const int room = TILE_LDS_BUDGET - tile_hist_bytes(B);
    uint32_t ch = 1024;
    while ((int)(2 * ch * sizeof(RecK)) <= room && (int)(2 * ch) <= tile)
        ch *= 2;
    return (int)(ch * sizeof(RecK)) <= room ? ch : 0;
}

// Tiles of a launch: the largest power-of-two tile (1024 threads times 4,
// 8 or 16 slots, at most ept_max) that still gives every CU one; then, when
// every tile keeps a dense table of more than twice its slots in buckets
// (dense_b buckets, 0 for local tables), larger tiles as long as half the
// CUs still get one (the tables' writes, column sums and reads grow with
// the tile count: a 128 x 128 grid steps in 65 us with 128 tiles of 8192
// slots, 75 us with 256 of 4096 and 80 us with 64 of 16384); then, when a launch needs
// more than one round of TILE_FILL tiles, a whole number of rounds of
// equal (even) slot counts, so that the last round is not a short tail.
static void choose_tiles(Plan *p, int64_t n_items, int ept_max, int64_t dense_b)
{
    auto tiles_for = [&](int e) {
        return (n_items + (int64_t)TILE_THREADS * e - 1) / ((int64_t)TILE_THREADS * e);
    };
    int ept = ept_max;
    while (ept > 4 && tiles_for(ept) < TILE_FILL)
        ept /= 2;
    while (ept < ept_max && dense_b + 1 > 2 * (int64_t)TILE_THREADS * ept &&
           tiles_for(2 * ept) >= TILE_FILL / 2)
        ept *= 2;
    const int64_t T = (int64_t)TILE_THREADS * ept;
    int64_t nt = std::max<int64_t>(1, (n_items + T - 1) / T);
    int64_t tile = T;
    if (nt > TILE_FILL) {
        nt = (nt + TILE_FILL - 1) / TILE_FILL * TILE_FILL;
        tile = (n_items + nt - 1) / nt;
        tile += tile & 1;
        nt = std::max<int64_t>(1, (n_items + tile - 1) / tile);
    }
    if (nt > MAX_TILES)
        throw HipError{hipErrorInvalidValue, "too many SD slots for one plan"};
    p->tile_ept = ept;
    p->tile = (int32_t)tile;
    p->n_tiles = (int32_t)nt;
}

static Plan *build_plan(sdm_ctx *ctx, int mode, int64_t n_items,
                        const std::vector<double> &expected, double bucket_target,
                        double group_target, const std::vector<uint32_t> *seg_off = nullptr,
                        int tile_ept_max = TILE_EPT_MAX)
{
    Plan *p = new Plan();
    try {
        (void)ctx;
        const int32_t C = (int32_t)expected.size();
        const bool batched = seg_off != nullptr;
        const int64_t max_b = batched ? MAX_B_BATCH : MAX_B;
        // the bucket table must fit the tile kernel's LDS histogram: coarser
        // buckets for plans with many SDs
        double target = bucket_target;
        for (;;) {
            int64_t nbk = 0;
            for (int32_t c = 0; c < C; ++c) {
                const double m = std::max(expected[c], 1.0);
                int h = 0;
                while (m / std::ldexp(1.0, h) > target && h < 20)
                    ++h;
                nbk += (int64_t)1 << h;
            }
            if (nbk <= max_b || target >= 1e12)
                break;
            target *= 2.0;
        }
        p->mode = mode;
        p->n_items = n_items;
        p->n_cell = C;
        std::vector<int32_t> cell_h(C), cell_bb(C + 1);
        std::vector<int32_t> bucket_cell;
        std::vector<uint8_t> sub_bits;
        std::vector<double> bucket_exp;
        // records per group thread: larger groups when a bucket alone
        // exceeds the usual group size
        double e_max = 0.0;
        for (int32_t c = 0; c < C; ++c) {
            const double m = std::max(expected[c], 1.0);
            int h = 0;
            while (m / std::ldexp(1.0, h) > target && h < 20)
                ++h;
            e_max = std::max(e_max, m / std::ldexp(1.0, h));
        }
        p->gept = e_max > group_target ? GROUP_EPT_L : GROUP_EPT_S;
        if (p->gept == GROUP_EPT_L)
            group_target *= (double)GROUP_EPT_L / GROUP_EPT_S;
        const int nsub_max = GROUP_THREADS * p->gept;  // sub-buckets per group
        int nsub_bits = 0;
        while ((2 << nsub_bits) <= nsub_max)
            ++nsub_bits;
        int32_t B = 0;
        for (int32_t c = 0; c < C; ++c) {
            const double m = std::max(expected[c], 1.0);
            int h = 0;
            while (m / std::ldexp(1.0, h) > target && h < 20)
                ++h;
            cell_h[c] = h;
            cell_bb[c] = B;
            const double e = m / std::ldexp(1.0, h);
            int u = 0;
            while (e / std::ldexp(1.0, u + 1) >= 1.0 && u < nsub_bits)
                ++u;
            // the group kernel finds the sub-bucket in the 24 key bits below
            // the bucket's (fused records)
            if (u > 24 || h > 29)
                throw HipError{hipErrorInvalidValue, "key bits of a bucket exceed the record"};
            for (int i = 0; i < (1 << h); ++i) {
                bucket_cell.push_back(c);
                sub_bits.push_back((uint8_t)u);
                bucket_exp.push_back(e);
                ++B;
                if (B > max_b)
                    throw HipError{hipErrorInvalidValue, "too many buckets for one plan"};
            }
        }
        cell_bb[C] = B;
        // groups: consecutive buckets with expected total <= GROUP_TARGET
        std::vector<int32_t> group_first, group_of_bucket(B);
        {
            int32_t b = 0;
            while (b < B) {
                group_first.push_back(b);
                double acc = 0;
                int nsub = 0, n = 0;
                while (b < B) {
                    const int ns = 1 << sub_bits[b];
                    if (n > 0 && (acc + bucket_exp[b] > group_target || n + 1 > MAXB ||
                                  nsub + ns > nsub_max))
                        break;
                    acc += bucket_exp[b];
                    nsub += ns;
                    group_of_bucket[b] = (int32_t)group_first.size() - 1;
                    ++n;
                    ++b;
                }
            }
            group_first.push_back(B);
        }
        // groups that begin at a cell's first bucket and end after a cell's
        // last one (then a group finds its cells' starts in its own columns)
        p->whole_cells = true;
        for (size_t gi = 0; gi + 1 < group_first.size(); ++gi) {
            const int32_t f = group_first[gi], l = group_first[gi + 1];
            if (cell_bb[bucket_cell[f]] != f || cell_bb[bucket_cell[l - 1] + 1] != l)
                p->whole_cells = false;
        }
        choose_tiles(p, n_items, tile_ept_max, batched ? 0 : B);
        p->B = B;
        p->lhist = B;
        std::vector<int32_t> t_lb, t_nb, bk_ta, bk_tc;
        std::vector<uint32_t> t_loff;
        int64_t n_off = (int64_t)p->n_tiles * (B + 1);
        if (batched) {
            // each tile's runs (first and last run meeting its slots) and
            // their bucket range; the local tables packed one after another
            const std::vector<uint32_t> &so = *seg_off;
            auto run_of = [&](uint32_t slot) {  // largest r with so[r] <= slot
                return (int32_t)(std::upper_bound(so.begin(), so.begin() + C, slot) - so.begin()) - 1;
            };
            t_lb.resize(p->n_tiles);
            t_nb.resize(p->n_tiles);
            t_loff.resize(p->n_tiles);
            int64_t acc = 0;
            int lmax = 0;
            for (int32_t t = 0; t < p->n_tiles; ++t) {
                const int64_t s0 = (int64_t)t * p->tile;
                const int64_t s1 = std::min<int64_t>(s0 + p->tile, n_items) - 1;
                const int32_t f = std::max(0, run_of((uint32_t)s0));
                const int32_t l = std::max(f, run_of((uint32_t)s1));
                t_lb[t] = cell_bb[f];
                t_nb[t] = cell_bb[l + 1] - cell_bb[f];
                t_loff[t] = (uint32_t)acc;
                acc += t_nb[t] + 1;
                lmax = std::max(lmax, t_nb[t]);
            }
            if (lmax >= (int)NO_BUCKET || acc >= ((int64_t)1 << 32))
                throw HipError{hipErrorInvalidValue, "a tile meets too many buckets"};
            n_off = acc;
            p->lhist = lmax;
            // bucket b: tiles wholly below it (their last bucket < b) and
            // tiles beginning below it; both nondecreasing in t
            bk_ta.resize(B + 1);
            bk_tc.resize(B + 1);
            int32_t ta = 0, tc = 0;
            for (int32_t b = 0; b <= B; ++b) {
                while (ta < p->n_tiles && t_lb[ta] + t_nb[ta] <= b)
                    ++ta;
                while (tc < p->n_tiles && t_lb[tc] < b)
                    ++tc;
                bk_ta[b] = ta;
                bk_tc[b] = tc;
            }
        }
        p->chunk = tile_chunk_for(p->lhist, p->tile);
        if (p->chunk == 0)
            throw HipError{hipErrorInvalidValue, "bucket table exceeds the tile LDS budget"};
        p->bucket_target = target;
        p->group_target = group_target;
        p->B = B;
        p->G = (int32_t)group_first.size() - 1;
        p->cell_h = upload(p, cell_h);
        p->cell_bucket_base = upload(p, cell_bb);
        p->bucket_cell = upload(p, bucket_cell);
        p->sub_bits = upload(p, sub_bits);
        p->group_first = upload(p, group_first);
        const bool fused = mode == MODE_FUSED;
        const size_t R = (size_t)p->n_tiles * p->tile;
        p->tile_off = (uint16_t *)dalloc(p, 2ull * (size_t)n_off);
        if (batched) {
            p->tile_lb = upload(p, t_lb);
            p->tile_nb = upload(p, t_nb);
            p->tile_loff = upload(p, t_loff);
            p->bk_ta = upload(p, bk_ta);
            p->bk_tc = upload(p, bk_tc);
        } else {
            p->tile_offT = (uint16_t *)dalloc(p, 2ull * (size_t)n_off);
        }
        if (fused) {
            p->rec_f = (uint64_t *)dalloc(p, sizeof(uint64_t) * R);
        } else {
            p->rec_k = (RecK *)dalloc(p, sizeof(RecK) * R);
        }
        p->n_acc = (uint32_t *)dalloc(p, 64);
        p->bucket_start = (uint32_t *)dalloc(p, 4ull * (B + 1));
        p->cell_start_ws = (uint32_t *)dalloc(p, 4ull * (C + 1));
        p->n_live_ws = (int64_t *)dalloc(p, 8);
        p->sk = (uint64_t *)dalloc(p, 16ull * n_items + 64);
        p->ss = (uint32_t *)dalloc(p, 8ull * n_items + 64);
        p->sb = (uint32_t *)dalloc(p, 8ull * n_items + 64);
        p->seam_open = (SeamRec *)dalloc(p, sizeof(SeamRec) * p->G);
        p->seam_close = (SeamRec *)dalloc(p, sizeof(SeamRec) * p->G);
        p->seam_state = (uint32_t *)dalloc(p, 4ull * p->G);
        p->group_tot = (uint32_t *)dalloc(p, 4ull * p->G);
        p->group_stats = (uint32_t *)dalloc(p, 20ull * p->G);
        SDM_HIP(hipMemset(p->n_acc, 0, 64));
        SDM_HIP(hipMemset(p->seam_state, 0, 4ull * p->G));
        SDM_HIP(hipMemset(p->group_tot, 0, 4ull * p->G));
        SDM_HIP(hipDeviceSynchronize());
    } catch (...) {
        free_plan(p);
        throw;
    }
    return p;
}

Plan *get_plan(sdm_ctx *ctx, int mode, int64_t n_items, int32_t n_cell,
               double expected_per_cell)
{
    if (expected_per_cell <= 0)
        expected_per_cell = (double)n_items / (double)std::max(n_cell, 1);
    PlanKey key{mode, n_items, n_cell, (int64_t)std::llround(expected_per_cell * 1000.0)};
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end())
        return it->second;
    std::vector<double> exp(n_cell, expected_per_cell);
    const double bt = ctx->dbg_bucket_target > 0 ? (double)ctx->dbg_bucket_target : BUCKET_TARGET;
    // small launches: smaller groups (at least two per CU where the buckets
    // allow), since parallelism, not per-group overhead, limits them
    const double gt = std::min(GROUP_TARGET, std::max(1024.0, (double)n_items / 512.0));
    Plan *p = build_plan(ctx, mode, n_items, exp, bt, gt);
    ctx->plans[key] = p;
    return p;
}

// Schedules the batch autotuner chooses from: (expected SDs per key bucket,
// expected SDs per group, largest tile-kernel slots per thread).  Results
// never depend on the choice; schedules that build the same plan for a
// batch are timed once.
static const double kSchedules[][3] = {
    {1024.0, 3100.0, 16}, {512.0, 3100.0, 16},  {2048.0, 3100.0, 16}, {256.0, 3100.0, 16},
    {1024.0, 2400.0, 16}, {512.0, 2400.0, 16},  {512.0, 1600.0, 16},  {4096.0, 3100.0, 16},
    {512.0, 3100.0, 8},   {1024.0, 3100.0, 8},  {512.0, 2400.0, 8},   {256.0, 2400.0, 16},
};
int n_schedules() { return (int)(sizeof(kSchedules) / sizeof(kSchedules[0])); }

PlanShape shape_of(const Plan *p)
{
    return PlanShape{p->B,        p->G,    p->tile,          p->n_tiles,      p->tile_ept,
                     p->gept,     p->chunk, p->bucket_target, p->group_target};
}

Plan *build_batch_plan(sdm_ctx *ctx, const std::vector<sdm_segment> &segs, int64_t n_items,
                       int schedule)
{
    std::vector<double> exp(segs.size());
    for (size_t i = 0; i < segs.size(); ++i)
        exp[i] = (double)segs[i].n_sd;
    double bt = kSchedules[schedule][0], gt = kSchedules[schedule][1];
    const int ept = (int)kSchedules[schedule][2];
    if (ctx->dbg_bucket_target > 0)
        bt = (double)ctx->dbg_bucket_target;
    const int C = (int)segs.size();
    std::vector<uint32_t> off(C + 1), len(C);
    for (int c = 0; c < C; ++c) {
        off[c] = (uint32_t)segs[c].offset;
        len[c] = (uint32_t)segs[c].n_sd;
    }
    off[C] = (uint32_t)n_items;
    Plan *p = build_plan(ctx, MODE_FUSED, n_items, exp, bt, gt, &off, ept);
    try {
        std::vector<int32_t> run(C), kidx(C);
        std::vector<double> dv(C);
        std::vector<KernelDesc> kernels(C);
        for (int c = 0; c < C; ++c) {
            run[c] = (int32_t)segs[c].run;
            dv[c] = segs[c].dv;
            kidx[c] = c;
            kernels[c] = kernel_desc(segs[c].kernel);
        }
        p->seg_off = upload(p, off);
        p->seg_len = upload(p, len);
        p->seg_run = upload(p, run);
        p->seg_kernel = upload(p, kidx);
        p->seg_dv = upload(p, dv);
        p->kernels = upload(p, kernels);
        SDM_HIP(hipDeviceSynchronize());
    } catch (...) {
        free_plan(p);
        throw;
    }
    return p;
}

template <int EPT, bool LIST>
static void launch_tile(int grid, size_t lds, hipStream_t stream, const TileArgs &ta)
{
    static bool attr_set = false;
    if (!attr_set) {
        SDM_HIP(hipFuncSetAttribute((const void *)k_tile<TILE_THREADS, EPT, LIST>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    TILE_LDS_BUDGET));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_tile<TILE_THREADS, EPT, LIST>), dim3(grid), dim3(TILE_THREADS), lds,
                       stream, ta);
}

template <bool LIST>
static void launch_tile_ept(int ept, int grid, size_t lds, hipStream_t stream, const TileArgs &ta)
{
    if (ept == 16)
        launch_tile<16, LIST>(grid, lds, stream, ta);
    else if (ept == 8)
        launch_tile<8, LIST>(grid, lds, stream, ta);
    else
        launch_tile<4, LIST>(grid, lds, stream, ta);
}

// The fused single-cell launches k_small takes: the Philox keys (no
// caller-given uniforms), no cell ids to check, at most SMALL_CAP slots.
static bool small_step(const Plan *p, const StepInputs &in)
{
    return p->mode == MODE_FUSED && !p->seg_off && p->n_cell == 1 && !in.cell_id && !in.u01 &&
           in.n_sd <= SMALL_CAP && in.n_attr >= 1;
}

void engine_run(sdm_ctx *ctx, Plan *p, const StepInputs &in, hipStream_t stream)
{
    const bool list = p->mode != MODE_FUSED;
    uint32_t *cell_start = in.cell_start ? in.cell_start : p->cell_start_ws;
    int64_t *n_live_out = in.n_live_out ? in.n_live_out : p->n_live_ws;
    auto mark = [&](int i) {
        if (in.events[i])
            SDM_HIP(hipEventRecord(in.events[i], stream));
    };
    if (small_step(p, in)) {
        SmallArgs sa{};
        sa.n_sd = in.n_sd;
        sa.xi = in.xi;
        sa.attr = in.attr;
        sa.n_attr = in.n_attr;
        sa.stride = in.stride;
        sa.seed = in.seed;
        sa.run = in.run;
        sa.step = in.step;
        sa.step_dev = in.step_dev;
        sa.step_advance = in.step_advance;
        sa.dt = in.dt;
        sa.dv_cell = in.dv_cell;
        sa.dv = in.dv;
        sa.kern = in.kern;
        sa.slot_cell_local = in.slot_cell_local ? 1 : 0;
        sa.idx_out = in.idx_out;
        sa.cell_start = cell_start;
        sa.n_live_out = n_live_out;
        sa.counters = in.counters;
        sa.gamma_out = in.gamma_out;
        mark(0);
        hipLaunchKernelGGL(k_small, dim3(1), dim3(SMALL_THREADS), 0, stream, sa);
        SDM_HIP(hipGetLastError());
        mark(1);
        mark(2);
        mark(3);
        return;
    }

    TileArgs ta{};
    ta.mode = p->mode;
    ta.n_sd = in.n_sd;
    ta.n_live_in = in.n_live_in;
    ta.idx_in = in.idx_in;
    ta.xi = in.xi;
    ta.v = in.attr;
    ta.cell_id = in.cell_id;
    ta.n_cell = p->n_cell;
    ta.u01 = in.u01;
    ta.seed = in.seed;
    ta.run = in.run;
    ta.step = in.step;
    ta.step_dev = in.step_dev;
    ta.key_shift = 53 - std::max(1, ceil_log2_u64((uint64_t)std::max<int64_t>(p->n_items, 2)));
    ta.cell_h = p->cell_h;
    ta.cell_bucket_base = p->cell_bucket_base;
    ta.B = p->B;
    ta.seg_off = p->seg_off;
    ta.seg_len = p->seg_len;
    ta.seg_run = p->seg_run;
    ta.tile_off = p->tile_off;
    ta.tile_slots = (uint32_t)p->tile;
    ta.tile_lb = p->tile_lb;
    ta.tile_nb = p->tile_nb;
    ta.tile_loff = p->tile_loff;
    ta.rec_k = p->rec_k;
    ta.rec_f = p->rec_f;
    ta.chunk = p->chunk;
    // a fused launch of one cell, or of groups of whole cells, with dense
    // tables and at most one tile per group thread: the group kernel sums
    // its bucket starts itself
    const bool direct = !list && (p->n_cell == 1 || p->whole_cells) && !p->tile_lb &&
                        p->n_tiles <= GROUP_THREADS;
    ta.start_zero = (p->n_tiles > 64 && !p->tile_lb && !direct) ? p->bucket_start : nullptr;
    ta.n_acc = p->n_acc;
    ta.err = ctx->err_dev;
    const size_t lds = (size_t)tile_hist_bytes(p->lhist) + (size_t)p->chunk * sizeof(RecK);
    mark(0);
    if (list)
        launch_tile_ept<true>(p->tile_ept, p->n_tiles, lds, stream, ta);
    else
        launch_tile_ept<false>(p->tile_ept, p->n_tiles, lds, stream, ta);
    SDM_HIP(hipGetLastError());
    if (p->tile_lb) {
        BatchScanArgs sa{};
        sa.tile_off = p->tile_off;
        sa.tile_loff = p->tile_loff;
        sa.tile_lb = p->tile_lb;
        sa.tile_nb = p->tile_nb;
        sa.bk_ta = p->bk_ta;
        sa.bk_tc = p->bk_tc;
        sa.n_tiles = p->n_tiles;
        sa.B = p->B;
        sa.bucket_start = p->bucket_start;
        hipLaunchKernelGGL((k_colsum_batch<256>), dim3((p->B + 1 + 255) / 256), dim3(256), 0,
                           stream, sa);
        SDM_HIP(hipGetLastError());
    } else if (!direct) {
        ScanArgs sa{};
        sa.tile_off = p->tile_off;
        sa.tile_offT = p->tile_offT;
        sa.n_tiles = p->n_tiles;
        sa.B = p->B;
        sa.bucket_start = p->bucket_start;
        hipLaunchKernelGGL((k_colsum<256>), dim3((p->B + 1 + 63) / 64, (p->n_tiles + 63) / 64),
                           dim3(256), 0, stream, sa);
        SDM_HIP(hipGetLastError());
    }

    GroupArgs ga{};
    ga.mode = p->mode;
    ga.direct = direct ? 1 : 0;
    ga.n_total = p->n_acc;
    ga.B = p->B;
    ga.n_tiles = p->n_tiles;
    ga.tile = p->tile;
    ga.n_cell = p->n_cell;
    ga.group_first = p->group_first;
    ga.bucket_cell = p->bucket_cell;
    ga.sub_bits = p->sub_bits;
    ga.cell_h = p->cell_h;
    ga.cell_bucket_base = p->cell_bucket_base;
    ga.tile_offT = p->tile_offT;
    ga.tile_off = p->tile_off;
    ga.tile_lb = p->tile_lb;
    ga.tile_nb = p->tile_nb;
    ga.tile_loff = p->tile_loff;
    ga.rec_k = p->rec_k;
    ga.rec_f = p->rec_f;
    ga.cell_id = in.cell_id;
    ga.bucket_start = p->bucket_start;
    ga.cell_start = cell_start;
    ga.sk = p->sk;
    ga.ss = p->ss;
    ga.sb = p->sb;
    ga.group_cap = ctx->dbg_group_cap;
    ga.idx_out = in.idx_out;
    ga.xi = in.xi;
    ga.attr = in.attr;
    ga.n_attr = in.n_attr;
    ga.stride = in.stride;
    ga.dt = in.dt;
    ga.dv_cell = in.dv_cell;
    ga.dv = in.dv;
    ga.kern = in.kern;
    ga.seg_off = p->seg_off;
    ga.seg_run = p->seg_run;
    ga.seg_kernel = p->seg_kernel;
    ga.seg_dv = p->seg_dv;
    ga.kernels = p->kernels;
    ga.seed = in.seed;
    ga.run = in.run;
    ga.step = in.step;
    ga.step_dev = in.step_dev;
    ga.slot_cell_local = in.slot_cell_local ? 1 : 0;
    ga.counters = in.counters;
    ga.gamma_out = in.gamma_out;
    ga.seam_open = p->seam_open;
    ga.seam_close = p->seam_close;
    ga.seam_state = p->seam_state;
    ga.group_tot = p->group_tot;
    ga.group_stats = p->group_stats;
    mark(1);
    const bool one = p->n_cell == 1;
    const bool whole = direct && !one;  // the instance for groups of whole cells
    if (p->gept == GROUP_EPT_L && !list && one)
        hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT_L, true, true>), dim3(p->G),
                           dim3(GROUP_THREADS), 0, stream, ga);
    else if (p->gept == GROUP_EPT_L && !list && whole)
        hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT_L, true, false, true>), dim3(p->G),
                           dim3(GROUP_THREADS), 0, stream, ga);
    else if (p->gept == GROUP_EPT_L && !list)
        hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT_L, true>), dim3(p->G),
                           dim3(GROUP_THREADS), 0, stream, ga);
    else if (p->gept == GROUP_EPT_L)
        hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT_L, false>), dim3(p->G),
                           dim3(GROUP_THREADS), 0, stream, ga);
    else if (!list && one)
        hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT_S, true, true>), dim3(p->G),
                           dim3(GROUP_THREADS), 0, stream, ga);
    else if (!list && whole)
        hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT_S, true, false, true>), dim3(p->G),
                           dim3(GROUP_THREADS), 0, stream, ga);
    else if (!list)
        hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT_S, true>), dim3(p->G),
                           dim3(GROUP_THREADS), 0, stream, ga);
    else
        hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT_S, false>), dim3(p->G),
                           dim3(GROUP_THREADS), 0, stream, ga);
    SDM_HIP(hipGetLastError());

    FinishArgs fa{};
    fa.mode = p->mode;
    fa.G = p->G;
    fa.n_cell = p->n_cell;
    fa.seam_open = p->seam_open;
    fa.seam_close = p->seam_close;
    fa.seam_state = p->seam_state;
    fa.group_tot = p->group_tot;
    fa.group_stats = p->group_stats;
    fa.xi = in.xi;
    fa.attr = in.attr;
    fa.n_attr = in.n_attr;
    fa.stride = in.stride;
    fa.dt = in.dt;
    fa.dv_cell = in.dv_cell;
    fa.dv = in.dv;
    fa.kern = in.kern;
    fa.seg_off = p->seg_off;
    fa.seg_run = p->seg_run;
    fa.seg_kernel = p->seg_kernel;
    fa.seg_dv = p->seg_dv;
    fa.kernels = p->kernels;
    fa.seed = in.seed;
    fa.run = in.run;
    fa.slot_cell_local = in.slot_cell_local ? 1 : 0;
    fa.counters = in.counters;
    fa.gamma_out = in.gamma_out;
    fa.n_acc = p->n_acc;
    fa.cell_start = cell_start;
    fa.n_live_out = n_live_out;
    fa.step_advance = in.step_advance;
    constexpr int FT = 256;
    const int grid3 = std::max(1, (p->G + FT - 1) / FT);
    mark(2);
    hipLaunchKernelGGL((k_finish<FT>), dim3(grid3), dim3(FT), 0, stream, fa);
    SDM_HIP(hipGetLastError());
    mark(3);
}

}  // namespace sdm
