// The backend API routines of the timestep workflow (arXiv:2101.06318,
// Sec. 3.2), one HIP kernel each, behind the C ABI of include/sdm.h.  These
// are the building blocks a caller composes step by step; the fused
// timestep (sdm_step) computes the same result in four kernels.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "sdm_internal.h"

using namespace sdm;

namespace {

constexpr int TPB = 256;

inline int blocks_for(int64_t n, int64_t per_block)
{
    return (int)std::max<int64_t>(1, (n + per_block - 1) / per_block);
}

// ----------------------------------------------------------------- urand
__global__ void k_urand(double *u01, int64_t n, uint64_t seed, uint32_t run,
                        uint32_t step, const uint32_t *step_dev, uint32_t stream_id)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = 2 * p;
    if (e >= n)
        return;
    const WordPair w = philox_words(seed, run, step_of(step, step_dev), stream_id, (uint64_t)p);
    u01[e] = word_to_uniform(w.even);
    if (e + 1 < n)
        u01[e + 1] = word_to_uniform(w.odd);
}

// ------------------------------------------------- remove_if_equal_0
constexpr int CMP_THREADS = 256;
constexpr int CMP_EPT = 8;
constexpr int CMP_TILE = CMP_THREADS * CMP_EPT;

__global__ void k_compact_count(const uint32_t *idx, const int64_t *n_live, int64_t cap,
                                const uint64_t *xi, uint32_t *tile_cnt)
{
    __shared__ uint32_t s;
    if (threadIdx.x == 0)
        s = 0;
    __syncthreads();
    const int64_t n = min(*n_live, cap);
    const int64_t base = (int64_t)blockIdx.x * CMP_TILE;
    uint32_t c = 0;
    for (int k = 0; k < CMP_EPT; ++k) {
        const int64_t i = base + (int64_t)k * CMP_THREADS + threadIdx.x;
        if (i < n && xi[idx[i]] > 0)
            ++c;
    }
    atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0)
        tile_cnt[blockIdx.x] = s;
}

__global__ void k_compact_scan(uint32_t *tile_cnt, int n_tiles, int64_t *n_live, int64_t cap)
{
    // single block: exclusive scan of the tile counts (serial per chunk)
    __shared__ uint32_t part[TPB + 1];
    const int chunk = (n_tiles + TPB - 1) / TPB;
    const int lo = min(n_tiles, (int)threadIdx.x * chunk), hi = min(n_tiles, lo + chunk);
    uint32_t sum = 0;
    for (int t = lo; t < hi; ++t)
        sum += tile_cnt[t];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < TPB; ++i) {
            const uint32_t v = part[i];
            part[i] = run;
            run += v;
        }
        part[TPB] = run;
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int t = lo; t < hi; ++t) {
        const uint32_t v = tile_cnt[t];
        tile_cnt[t] = run;
        run += v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        tile_cnt[n_tiles] = (uint32_t)min(*n_live, cap);  // old count, read by the scatter
        *n_live = (int64_t)part[TPB];
    }
}

__global__ void k_compact_scatter(const uint32_t *idx, const uint32_t *tile_cnt, int n_tiles,
                                  const uint64_t *xi, uint32_t *tmp)
{
    // stable within the tile: thread-major order k*THREADS + tid is the
    // original order, so rank = count of kept items before it in that order.
    __shared__ uint32_t flags[CMP_TILE];
    __shared__ uint32_t scan[CMP_TILE + 1];
    const int64_t n = tile_cnt[n_tiles];
    const int64_t base = (int64_t)blockIdx.x * CMP_TILE;
    for (int k = 0; k < CMP_EPT; ++k) {
        const int li = k * CMP_THREADS + threadIdx.x;
        const int64_t i = base + li;
        flags[li] = (i < n && xi[idx[i]] > 0) ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < CMP_TILE; ++i) {
            scan[i] = run;
            run += flags[i];
        }
        scan[CMP_TILE] = run;
    }
    __syncthreads();
    const uint32_t off = tile_cnt[blockIdx.x];
    for (int k = 0; k < CMP_EPT; ++k) {
        const int li = k * CMP_THREADS + threadIdx.x;
        if (flags[li])
            tmp[off + scan[li]] = idx[base + li];
    }
}

__global__ void k_copy_u32(uint32_t *dst, const uint32_t *src, const int64_t *n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *n)
        dst[i] = src[i];
}

// ----------------------------------------------------------- flag_pairs
__device__ __forceinline__ int32_t cell_of(const int32_t *cell_id, uint32_t s)
{
    return cell_id ? cell_id[s] : 0;
}

__global__ void k_flag_pairs(uint8_t *flag, const int32_t *cell_id, const uint32_t *cell_start,
                             const uint32_t *idx, const int64_t *n_live)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = *n_live;
    if (i >= n)
        return;
    const int32_t c = cell_of(cell_id, idx[i]);
    uint8_t f = 0;
    if (i + 1 < n && cell_of(cell_id, idx[i + 1]) == c &&
        ((i - (int64_t)cell_start[c]) & 1) == 0)
        f = 1;
    flag[i] = f;
}

// Flagged opener of slot q, or -1.
__device__ __forceinline__ int64_t opener_of_slot(const uint8_t *flag, int64_t q, int64_t n)
{
    const int64_t i = 2 * q;
    if (flag[i])
        return i;
    if (i + 1 < n && flag[i + 1])
        return i + 1;
    return -1;
}

enum { PR_KERNEL = 1, PR_MAX = 2, PR_NORM = 4 };

// coalescence_kernel / times_max / normalize / pair_rate in one kernel body:
// `which` selects the factors applied (PR_KERNEL overwrites, the others
// multiply in place), in the order of eq. (3).
__global__ void k_pair_rate(double *pair_prob, int which, const uint8_t *flag,
                            const double *volume, const uint64_t *xi, double dt,
                            const double *dv_cell, const int32_t *cell_id,
                            const uint32_t *cell_start, const uint32_t *idx,
                            const int64_t *n_live, KernelDesc kd)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = *n_live;
    if (q >= n / 2)
        return;
    const int64_t i = opener_of_slot(flag, q, n);
    if (i < 0) {
        if (which & PR_KERNEL)
            pair_prob[q] = 0.0;
        return;
    }
    const uint32_t j = idx[i], k = idx[i + 1];
    double p = (which & PR_KERNEL) ? kernel_value(kd, volume[j], volume[k]) : pair_prob[q];
    if (which & PR_MAX) {
        const uint64_t a = xi[j], b = xi[k];
        p = p * (double)(a > b ? a : b);
    }
    if (which & PR_NORM) {
        const int32_t c = cell_of(cell_id, j);
        const uint64_t n_c = (uint64_t)(cell_start[c + 1] - cell_start[c]);
        const double norm = (dt / dv_cell[c]) * (double)pair_scale(n_c);
        p = p * norm;
    }
    pair_prob[q] = p;
}

__global__ void k_compute_gamma(double *pair_prob, const double *u01, uint64_t seed,
                                uint32_t run, uint32_t step, const uint32_t *step_dev,
                                const int64_t *n_live)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_slot = *n_live / 2;
    const int64_t q0 = 2 * m;
    if (q0 >= n_slot)
        return;
    double phi0, phi1;
    if (u01) {
        phi0 = u01[q0];
        phi1 = q0 + 1 < n_slot ? u01[q0 + 1] : 0.0;
    } else {
        const WordPair w = philox_words(seed, run, step_of(step, step_dev), SDM_STREAM_GAMMA,
                                        (uint64_t)m);
        phi0 = word_to_uniform(w.even);
        phi1 = word_to_uniform(w.odd);
    }
    pair_prob[q0] = ceil(pair_prob[q0] - phi0);
    if (q0 + 1 < n_slot)
        pair_prob[q0 + 1] = ceil(pair_prob[q0 + 1] - phi1);
}

__global__ void k_update(uint64_t *xi, double *attr, int32_t n_attr, int64_t stride,
                         const double *gamma, const uint8_t *flag, const uint32_t *idx,
                         const int64_t *n_live, uint64_t *counters)
{
    __shared__ uint32_t red[5 * (TPB / 64) + 8];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = *n_live;
    Stats st{0, 0, 0, 0, 0};
    if (q < n / 2) {
        const int64_t i = opener_of_slot(flag, q, n);
        if (i >= 0) {
            const uint32_t a = idx[i], b = idx[i + 1];
            const Collision c = collide(xi[a], xi[b], gamma[q], st);
            if (c.g)
                apply_collision(c, a, b, xi, attr, n_attr, stride);
        }
    }
    flush_stats<TPB>(st, counters, red);
}

// ------------------------------------------------------------- moments
__global__ void k_moments(double *M, const uint64_t *xi, const double *v, const uint32_t *idx,
                          const uint32_t *cell_start, const double *dv_cell, double dv)
{
    __shared__ double red[3][TPB];
    const int c = blockIdx.x;
    const uint32_t lo = cell_start[c], hi = cell_start[c + 1];
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += TPB) {
        const uint32_t s = idx[i];
        const double x = (double)xi[s];
        const double xv = x * v[s];
        m0 = m0 + x;
        m1 = m1 + xv;
        m2 = m2 + xv * v[s];
    }
    red[0][threadIdx.x] = m0;
    red[1][threadIdx.x] = m1;
    red[2][threadIdx.x] = m2;
    __syncthreads();
    for (int o = TPB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] = red[0][threadIdx.x] + red[0][threadIdx.x + o];
            red[1][threadIdx.x] = red[1][threadIdx.x] + red[1][threadIdx.x + o];
            red[2][threadIdx.x] = red[2][threadIdx.x] + red[2][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double d = dv_cell ? dv_cell[c] : dv;
        M[3 * c] = red[0][0] / d;
        M[3 * c + 1] = red[1][0] / d;
        M[3 * c + 2] = red[2][0] / d;
    }
}

__global__ void k_reassign(int32_t *cell_id, int64_t n_sd, int32_t n_cell, uint64_t seed,
                           uint32_t step, const uint32_t *step_dev)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = 2 * p;
    if (e >= n_sd)
        return;
    const WordPair w = philox_words(seed, 0, step_of(step, step_dev), SDM_STREAM_REASSIGN,
                                    (uint64_t)p);
    cell_id[e] = (int32_t)(word_to_uniform(w.even) * (double)n_cell);
    if (e + 1 < n_sd)
        cell_id[e + 1] = (int32_t)(word_to_uniform(w.odd) * (double)n_cell);
}

// ------------------------------------------------ O(n) permutations
// The per-cell permutations the paper names besides sorting by random keys
// (Sec. 3.2): the serial O(n) permutation of its CPU backend (Fisher-Yates)
// and MergeShuffle.  Both permute each cell's segment of a cell-sorted
// Index in place; every random draw is the Philox word of its global
// position in a stream of its own, so results do not depend on the launch.
constexpr uint32_t STREAM_FY = 5;
constexpr uint32_t STREAM_MERGE = 8;
constexpr int MERGE_BLOCK = 16;

// Uniform integer in [0, m): floor(U m) = (w m) >> 53, w the 53-bit word.
__device__ __forceinline__ uint64_t draw_below(uint64_t seed, uint32_t run, uint32_t step,
                                               uint32_t stream, uint64_t e, uint64_t m)
{
    const uint64_t w = philox_word(seed, run, step, stream, e) >> 11;
    return __umul64hi(w << 11, m);
}

__device__ __forceinline__ void fy_range(uint32_t *idx, int64_t s, int64_t e, uint64_t seed,
                                         uint32_t run, uint32_t step)
{
    for (int64_t i = e - 1; i > s; --i) {
        const int64_t k =
            s + (int64_t)draw_below(seed, run, step, STREAM_FY, (uint64_t)i, (uint64_t)(i - s + 1));
        const uint32_t a = idx[i], b = idx[k];
        idx[i] = b;
        idx[k] = a;
    }
}

// Cell containing sorted position p: largest c with cell_start[c] <= p.
__device__ __forceinline__ int cell_of_position(const uint32_t *cs, int n_cell, uint32_t p)
{
    int lo = 0, hi = n_cell;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cs[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ void k_fisher_yates(uint32_t *idx, const uint32_t *cs, int n_cell, uint64_t seed,
                               uint32_t run, uint32_t step, const uint32_t *step_dev)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cell)
        return;
    fy_range(idx, cs[c], cs[c + 1], seed, run, step_of(step, step_dev));
}

// Level 0: Fisher-Yates on every block of MERGE_BLOCK positions from a
// cell's start.  Level d >= 1: the pairwise merges of blocks of
// MERGE_BLOCK 2^(d-1) positions.  One thread per position; the thread at a
// block (or merge) start does it.
__global__ void k_merge_level(uint32_t *idx, const uint32_t *cs, int n_cell, const int64_t *n_live,
                              int d, uint64_t seed, uint32_t run, uint32_t step,
                              const uint32_t *step_dev)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= *n_live)
        return;
    const int c = cell_of_position(cs, n_cell, (uint32_t)p);
    const int64_t c0 = cs[c], c1 = cs[c + 1];
    const uint32_t t = step_of(step, step_dev);
    if (d == 0) {
        if ((p - c0) % MERGE_BLOCK == 0)
            fy_range(idx, p, min(p + MERGE_BLOCK, c1), seed, run, t);
        return;
    }
    const int64_t w = (int64_t)MERGE_BLOCK << (d - 1);
    if ((p - c0) % (2 * w) != 0 || p + w >= c1)
        return;
    const int64_t s = p, m = p + w, e = min(p + 2 * w, c1);
    const uint32_t sc = STREAM_MERGE + 2u * (uint32_t)d;
    int64_t i = s, j = m;
    for (;;) {
        const uint64_t coin = philox_word(seed, run, t, sc, (uint64_t)i) >> 63;
        if (coin == 0) {
            if (i == j)
                break;
        } else {
            if (j == e)
                break;
            const uint32_t a = idx[i], b = idx[j];
            idx[i] = b;
            idx[j] = a;
            ++j;
        }
        ++i;
    }
    for (; i < e; ++i) {
        const int64_t k = s + (int64_t)draw_below(seed, run, t, sc + 1u, (uint64_t)i,
                                                  (uint64_t)(i - s + 1));
        const uint32_t a = idx[i], b = idx[k];
        idx[i] = b;
        idx[k] = a;
    }
}

}  // namespace

// ====================================================================== ABI
// Step 0 as four launches over an Index of capacity cap: per-tile live
// counts, their scan (which also updates *n_live), the stable scatter into
// tmp, and the copy back.  tmp holds cap + 64 ids, tile_cnt
// blocks_for(cap, CMP_TILE) + 1 words.
static void launch_compaction(uint32_t *idx, int64_t *n_live, int64_t cap, const uint64_t *xi,
                              uint32_t *tmp, uint32_t *tile_cnt, hipStream_t stream)
{
    const int n_tiles = blocks_for(cap, CMP_TILE);
    hipLaunchKernelGGL(k_compact_count, dim3(n_tiles), dim3(CMP_THREADS), 0, stream, idx,
                       n_live, cap, xi, tile_cnt);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(TPB), 0, stream, tile_cnt, n_tiles, n_live,
                       cap);
    hipLaunchKernelGGL(k_compact_scatter, dim3(n_tiles), dim3(CMP_THREADS), 0, stream, idx,
                       tile_cnt, n_tiles, xi, tmp);
    hipLaunchKernelGGL(k_copy_u32, dim3(blocks_for(cap, TPB)), dim3(TPB), 0, stream, idx, tmp,
                       n_live);
    SDM_HIP(hipGetLastError());
}

// Fixed scratch of sdm_remove_if_equal_0_noalloc, for callers that cannot
// allocate: the compacted ids (SDM_NOALLOC_MAX_IDS + 64 words), then the
// per-tile counts.  Every GPU the library runs on holds its own copy for the
// life of the process.  In host code `scratch` names a host-side stand-in,
// never the device memory: kernels receive the address that
// hipGetSymbolAddress returns for the current device.
constexpr int64_t NOALLOC_IDS_WORDS = SDM_NOALLOC_MAX_IDS + 64;
constexpr int64_t NOALLOC_TILE_WORDS = (SDM_NOALLOC_MAX_IDS + CMP_TILE - 1) / CMP_TILE + 64;
static __device__ __align__(256) uint32_t scratch[NOALLOC_IDS_WORDS + NOALLOC_TILE_WORDS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static uint32_t *g_scratch_dev[NOALLOC_MAX_DEVICES];

// Device address of `scratch` on the current device, resolved once per
// device with that device current.
static int noalloc_scratch(uint32_t **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(SDM_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(SDM_E_UNSUPPORTED, "device %d beyond the %d the scratch table covers", dev,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SDM_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<uint32_t *>(p);
    }
    *out = g_scratch_dev[dev];
    return SDM_OK;
}

extern "C" {

int sdm_urand(sdm_ctx *ctx, double *u01, int64_t n, const sdm_rng *rng, uint32_t stream_id,
              hipStream_t stream)
{
    REQUIRE(ctx && rng, "ctx/rng is NULL");
    REQUIRE(n >= 0, "n < 0");
    if (n == 0)
        return SDM_OK;
    REQUIRE(u01, "u01 is NULL");
    REQUIRE(n <= (int64_t)1 << 33, "n too large for the 32-bit counter word");
    SDM_TRY
    hipLaunchKernelGGL(k_urand, dim3(blocks_for((n + 1) / 2, TPB)), dim3(TPB), 0, stream, u01, n,
                       rng->seed, rng->run, rng->step, rng->step_dev, stream_id);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_remove_if_equal_0(sdm_ctx *ctx, uint32_t *idx, int64_t *n_live_dev, const uint64_t *xi,
                          hipStream_t stream)
{
    REQUIRE(ctx && idx && n_live_dev && xi, "null argument");
    SDM_TRY
    const int n_tiles = blocks_for(ctx->n_sd_max, CMP_TILE);
    launch_compaction(idx, n_live_dev, ctx->n_sd_max, xi, ctx->tmp_u32, ctx->tile_cnt, stream);
    SDM_CATCH
}

int sdm_remove_if_equal_0_noalloc(uint32_t *idx, int64_t *n_live_dev, const uint64_t *xi,
                                  int64_t n_sd_max, hipStream_t stream)
{
    REQUIRE(idx && n_live_dev && xi, "null argument");
    REQUIRE(n_sd_max >= 1 && n_sd_max <= SDM_NOALLOC_MAX_IDS,
            "n_sd_max = %lld outside [1, %lld] (the fixed scratch holds SDM_NOALLOC_MAX_IDS ids)",
            (long long)n_sd_max, (long long)SDM_NOALLOC_MAX_IDS);
    uint32_t *ws = nullptr;
    const int rc = noalloc_scratch(&ws);
    if (rc != SDM_OK)
        return rc;
    SDM_TRY
    launch_compaction(idx, n_live_dev, n_sd_max, xi, ws, ws + NOALLOC_IDS_WORDS, stream);
    SDM_CATCH
}

int sdm_cell_sort(sdm_ctx *ctx, uint32_t *cell_start, uint32_t *idx, const int64_t *n_live_dev,
                  const int32_t *cell_id, int32_t n_cell, hipStream_t stream)
{
    REQUIRE(ctx && cell_start && idx && n_live_dev, "null argument");
    REQUIRE(n_cell >= 1 && n_cell <= ctx->n_cell_max, "n_cell out of range");
    SDM_TRY
    Plan *p = get_plan(ctx, MODE_CELLSORT, ctx->n_sd_max, n_cell, 0.0);
    StepInputs in;
    in.n_live_in = n_live_dev;
    in.idx_in = idx;
    in.cell_id = cell_id;
    in.idx_out = ctx->tmp_u32;
    in.cell_start = cell_start;
    in.n_live_out = p->n_live_ws;
    engine_run(ctx, p, in, stream);
    hipLaunchKernelGGL(k_copy_u32, dim3(blocks_for(ctx->n_sd_max, TPB)), dim3(TPB), 0, stream,
                       idx, ctx->tmp_u32, n_live_dev);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_shuffle_per_cell(sdm_ctx *ctx, uint32_t *cell_start, uint32_t *idx,
                         const int64_t *n_live_dev, const int32_t *cell_idx,
                         const int32_t *cell_id, int32_t n_cell, const double *u01_by_sd,
                         const sdm_rng *rng, hipStream_t stream)
{
    REQUIRE(ctx && cell_start && idx && n_live_dev, "null argument");
    REQUIRE(n_cell >= 1 && n_cell <= ctx->n_cell_max, "n_cell out of range");
    REQUIRE(u01_by_sd || rng, "need u01_by_sd or rng");
    (void)cell_idx;  // traversal order hint: the schedule here is the plan's
    SDM_TRY
    Plan *p = get_plan(ctx, MODE_SHUFFLE, ctx->n_sd_max, n_cell, 0.0);
    StepInputs in;
    in.n_live_in = n_live_dev;
    in.idx_in = idx;
    in.cell_id = cell_id;
    in.u01 = u01_by_sd;
    if (rng) {
        in.seed = rng->seed;
        in.run = rng->run;
        in.step = rng->step;
        in.step_dev = rng->step_dev;
    }
    in.idx_out = ctx->tmp_u32;
    in.cell_start = cell_start;
    in.n_live_out = p->n_live_ws;
    engine_run(ctx, p, in, stream);
    hipLaunchKernelGGL(k_copy_u32, dim3(blocks_for(ctx->n_sd_max, TPB)), dim3(TPB), 0, stream,
                       idx, ctx->tmp_u32, n_live_dev);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_shuffle_variant(sdm_ctx *ctx, int32_t method, uint32_t *cell_start, uint32_t *idx,
                        const int64_t *n_live_dev, const int32_t *cell_id, int32_t n_cell,
                        const sdm_rng *rng, hipStream_t stream)
{
    REQUIRE(method == SDM_SHUFFLE_FISHER_YATES || method == SDM_SHUFFLE_MERGE,
            "unknown shuffle method %d", method);
    REQUIRE(rng, "rng is NULL");
    REQUIRE(ctx && cell_start && idx && n_live_dev, "null argument");
    REQUIRE(ctx->n_sd_max <= ((int64_t)1 << 32), "positions must fit the Philox element word");
    if (int rc = sdm_cell_sort(ctx, cell_start, idx, n_live_dev, cell_id, n_cell, stream))
        return rc;
    SDM_TRY
    if (method == SDM_SHUFFLE_FISHER_YATES) {
        hipLaunchKernelGGL(k_fisher_yates, dim3(blocks_for(n_cell, 64)), dim3(64), 0, stream, idx,
                           cell_start, n_cell, rng->seed, rng->run, rng->step, rng->step_dev);
    } else {
        // levels until a block spans the largest possible cell
        int levels = 1;
        while (((int64_t)MERGE_BLOCK << (levels - 1)) < ctx->n_sd_max)
            ++levels;
        for (int d = 0; d < levels; ++d)
            hipLaunchKernelGGL(k_merge_level, dim3(blocks_for(ctx->n_sd_max, TPB)), dim3(TPB), 0,
                               stream, idx, cell_start, n_cell, n_live_dev, d, rng->seed,
                               rng->run, rng->step, rng->step_dev);
    }
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_flag_pairs(sdm_ctx *ctx, uint8_t *pair_flag, const int32_t *cell_id,
                   const int32_t *cell_idx, const uint32_t *cell_start, const uint32_t *idx,
                   const int64_t *n_live_dev, hipStream_t stream)
{
    REQUIRE(ctx && pair_flag && cell_start && idx && n_live_dev, "null argument");
    (void)cell_idx;
    SDM_TRY
    hipLaunchKernelGGL(k_flag_pairs, dim3(blocks_for(ctx->n_sd_max, TPB)), dim3(TPB), 0, stream,
                       pair_flag, cell_id, cell_start, idx, n_live_dev);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

static int pair_rate_common(sdm_ctx *ctx, double *pair_prob, int which, const uint8_t *flag,
                            const double *volume, const uint64_t *xi, double dt,
                            const double *dv_cell, const int32_t *cell_id,
                            const uint32_t *cell_start, const uint32_t *idx,
                            const int64_t *n_live, const sdm_kernel *k, hipStream_t stream)
{
    KernelDesc kd{};
    if (which & PR_KERNEL) {
        REQUIRE(k, "kernel is NULL");
        if (int rc = check_kernel(*k, "kernel"))
            return rc;
        kd = kernel_desc(*k);
        REQUIRE(volume, "volume is NULL");
    }
    if (which & PR_MAX)
        REQUIRE(xi, "xi is NULL");
    if (which & PR_NORM)
        REQUIRE(dv_cell && cell_start, "dv_per_cell/cell_start is NULL");
    REQUIRE(ctx && pair_prob && flag && idx && n_live, "null argument");
    SDM_TRY
    hipLaunchKernelGGL(k_pair_rate, dim3(blocks_for(ctx->n_sd_max / 2 + 1, TPB)), dim3(TPB), 0,
                       stream, pair_prob, which, flag, volume, xi, dt, dv_cell, cell_id,
                       cell_start, idx, n_live, kd);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_coalescence_kernel(sdm_ctx *ctx, double *pair_prob, const uint8_t *pair_flag,
                           const double *volume, const uint32_t *idx, const int64_t *n_live_dev,
                           const sdm_kernel *kernel, hipStream_t stream)
{
    return pair_rate_common(ctx, pair_prob, PR_KERNEL, pair_flag, volume, nullptr, 0.0, nullptr,
                            nullptr, nullptr, idx, n_live_dev, kernel, stream);
}

int sdm_times_max(sdm_ctx *ctx, double *pair_prob, const uint64_t *xi, const uint8_t *pair_flag,
                  const uint32_t *idx, const int64_t *n_live_dev, hipStream_t stream)
{
    return pair_rate_common(ctx, pair_prob, PR_MAX, pair_flag, nullptr, xi, 0.0, nullptr,
                            nullptr, nullptr, idx, n_live_dev, nullptr, stream);
}

int sdm_normalize(sdm_ctx *ctx, double *pair_prob, double dt, const double *dv_per_cell,
                  const int32_t *cell_id, const int32_t *cell_idx, const uint32_t *cell_start,
                  const uint8_t *pair_flag, const uint32_t *idx, const int64_t *n_live_dev,
                  hipStream_t stream)
{
    (void)cell_idx;
    return pair_rate_common(ctx, pair_prob, PR_NORM, pair_flag, nullptr, nullptr, dt,
                            dv_per_cell, cell_id, cell_start, idx, n_live_dev, nullptr, stream);
}

int sdm_pair_rate(sdm_ctx *ctx, double *pair_prob, double dt, const double *dv_per_cell,
                  const uint8_t *pair_flag, const double *volume, const uint64_t *xi,
                  const int32_t *cell_id, const uint32_t *cell_start, const uint32_t *idx,
                  const int64_t *n_live_dev, const sdm_kernel *kernel, hipStream_t stream)
{
    return pair_rate_common(ctx, pair_prob, PR_KERNEL | PR_MAX | PR_NORM, pair_flag, volume, xi,
                            dt, dv_per_cell, cell_id, cell_start, idx, n_live_dev, kernel,
                            stream);
}

int sdm_compute_gamma(sdm_ctx *ctx, double *pair_prob, const double *u01_by_slot,
                      const sdm_rng *rng, const int64_t *n_live_dev, hipStream_t stream)
{
    REQUIRE(ctx && pair_prob && n_live_dev, "null argument");
    REQUIRE(u01_by_slot || rng, "need u01_by_slot or rng");
    SDM_TRY
    sdm_rng r{};
    if (rng)
        r = *rng;
    hipLaunchKernelGGL(k_compute_gamma, dim3(blocks_for(ctx->n_sd_max / 4 + 1, TPB)), dim3(TPB),
                       0, stream, pair_prob, u01_by_slot, r.seed, r.run, r.step, r.step_dev,
                       n_live_dev);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_update_attributes(sdm_ctx *ctx, uint64_t *xi, double *attr, int32_t n_attr,
                          int64_t attr_stride, const double *gamma, const uint8_t *pair_flag,
                          const uint32_t *idx, const int64_t *n_live_dev, uint64_t *counters_dev,
                          hipStream_t stream)
{
    REQUIRE(ctx && xi && gamma && pair_flag && idx && n_live_dev, "null argument");
    REQUIRE(n_attr >= 0 && n_attr <= ctx->n_attr_max, "n_attr out of range");
    REQUIRE(n_attr == 0 || (attr && attr_stride >= 1), "attr/stride invalid");
    SDM_TRY
    hipLaunchKernelGGL(k_update, dim3(blocks_for(ctx->n_sd_max / 2 + 1, TPB)), dim3(TPB), 0,
                       stream, xi, attr, n_attr, attr_stride, gamma, pair_flag, idx, n_live_dev,
                       counters_dev);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_moments(sdm_ctx *ctx, double *M, const uint64_t *xi, const double *volume,
                const uint32_t *idx, const uint32_t *cell_start, int32_t n_cell,
                const double *dv_per_cell, double dv, hipStream_t stream)
{
    REQUIRE(ctx && M && xi && volume && idx && cell_start, "null argument");
    REQUIRE(n_cell >= 1, "n_cell < 1");
    REQUIRE(dv_per_cell || dv > 0, "need dv_per_cell or dv > 0");
    SDM_TRY
    hipLaunchKernelGGL(k_moments, dim3(n_cell), dim3(TPB), 0, stream, M, xi, volume, idx,
                       cell_start, dv_per_cell, dv);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_reassign(sdm_ctx *ctx, int32_t *cell_id, int64_t n_sd, int32_t n_cell,
                 const sdm_rng *rng, hipStream_t stream)
{
    REQUIRE(ctx && cell_id && rng, "null argument");
    REQUIRE(n_cell >= 1 && (n_cell & (n_cell - 1)) == 0, "n_cell must be a power of two");
    REQUIRE(n_sd >= 0 && n_sd <= ctx->n_sd_max, "n_sd out of range");
    if (n_sd == 0)
        return SDM_OK;
    SDM_TRY
    hipLaunchKernelGGL(k_reassign, dim3(blocks_for((n_sd + 1) / 2, TPB)), dim3(TPB), 0, stream,
                       cell_id, n_sd, n_cell, rng->seed, rng->step, rng->step_dev);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

}  // extern "C"
