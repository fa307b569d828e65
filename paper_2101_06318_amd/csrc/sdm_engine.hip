// Bucketed segmented sort + pair pass: the fused SDM timestep on gfx950.
//
// Step 1 of the paper (Sec. 2.2, Sec. 3.2) orders each cell's live SDs by a
// random key (the GPU strategy of the paper: a sort with random keys) and
// pairs neighbours; Steps 2-3 evaluate eq. (3), gamma and eqs. (4)-(6) per
// pair.  The data path here streams the state once:
//
//  k_scatter  (one pass over the SD slots, coalesced): liveness (Step 0:
//             xi > 0), Philox shuffle key, bucket = (cell, top key bits);
//             the record (key, s, xi, v) is appended to its bucket's region.
//             Per-tile LDS histograms make one global atomic per
//             (tile, bucket).  The last workgroup scans the bucket counts
//             into ranks and cell_start.
//  k_group    one workgroup per group of consecutive buckets: LDS counting
//             sort by the next key bits, exact rank inside each sub-bucket
//             by (key, s) comparisons, then idx, the pair probabilities,
//             gamma and the collision update, written back only for pairs
//             that collide.  Pairs that straddle two groups leave a seam
//             record.
//  k_seams    the straddling pairs, counters, and bookkeeping for the next
//             launch.
//
// Oversized buckets (more records than their region) spill to an overflow
// list and their group is sorted by a global-memory bitonic network instead
// of in LDS; that path is exact, only slower, and practically never taken
// for i.i.d. keys.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>

#include "sdm_internal.h"

namespace sdm {

constexpr int SCATTER_THREADS = 1024;
constexpr int SCATTER_EPT = 8;       // items per thread (even)
constexpr int GROUP_THREADS = 512;
constexpr int GROUP_EPT = 6;
constexpr int GROUP_CAP = GROUP_THREADS * GROUP_EPT;
constexpr int MAXB = 256;            // buckets per group
constexpr int NSUB = 1024;           // sub-buckets per group
constexpr int LDS_BINS_MAX = 16384;  // scatter histogram (64 KiB)
constexpr double BUCKET_TARGET = 2048.0;
constexpr double GROUP_TARGET = 2048.0;
constexpr uint32_t NO_BUCKET = 0xFFFFFFFFu;

// ------------------------------------------------------------------ args
struct ScatterArgs {
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
    const uint32_t *slot_base;
    int32_t B;
    int32_t lds_bins;
    const uint32_t *seg_off;
    const int32_t *seg_run;
    uint32_t *cursor;
    uint64_t *rec_key;
    uint32_t *rec_s;
    uint64_t *rec_xi;
    double *rec_v;
    uint32_t *ov_count;
    uint64_t *ov_key;
    uint32_t *ov_s;
    uint32_t *ov_bucket;
    uint32_t *rank_off;
    uint32_t *cell_start;
    int64_t *n_live_out;
    uint32_t *ticket;
    uint32_t *err;
};

struct GroupArgs {
    int mode;
    const int32_t *group_first;
    const int32_t *bucket_cell;
    const uint32_t *slot_base;
    const uint8_t *sub_bits;
    const int32_t *cell_h;
    uint32_t *cursor;
    const uint32_t *rank_off;
    const uint32_t *cell_start;
    const uint64_t *rec_key;
    const uint32_t *rec_s;
    const uint64_t *rec_xi;
    const double *rec_v;
    const uint32_t *ov_count;
    const uint64_t *ov_key;
    const uint32_t *ov_s;
    const uint32_t *ov_bucket;
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
};

struct SeamArgs {
    int mode;
    int32_t G;
    const SeamRec *seam_open;
    const SeamRec *seam_close;
    const uint32_t *seam_state;
    const uint32_t *group_tot;
    const uint32_t *cell_start;
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
    uint32_t *ov_count;
    uint32_t *ticket;
    uint32_t *step_advance;
};

// --------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t load_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Segment (run) containing SD slot s: largest r with seg_off[r] <= s.
__device__ __forceinline__ int find_seg(const uint32_t *seg_off, int n, uint32_t s)
{
    int lo = 0, hi = n;  // seg_off[n] > s
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg_off[mid] <= s)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Exclusive scan over THREADS values held one per thread; returns this
// thread's exclusive prefix and the total in *total.
template <int THREADS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *scratch,
                                                         uint32_t *total)
{
    constexpr int W = THREADS / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        scratch[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < W; ++w) {
            const uint32_t t = scratch[w];
            scratch[w] = run;
            run += t;
        }
        scratch[W] = run;
    }
    __syncthreads();
    const uint32_t res = scratch[wid] + x - v;
    *total = scratch[W];
    __syncthreads();
    return res;
}

// ------------------------------------------------------------- k_scatter
template <int THREADS, int EPT>
__global__ __launch_bounds__(THREADS) void k_scatter(ScatterArgs a)
{
    extern __shared__ uint32_t hist[];
    __shared__ uint32_t scan_scratch[THREADS / 64 + 1];
    __shared__ int s_last;
    const int tid = threadIdx.x;
    for (int i = tid; i < a.lds_bins; i += THREADS)
        hist[i] = 0;
    __syncthreads();

    const uint32_t step = step_of(a.step, a.step_dev);
    const bool fused = a.mode == MODE_FUSED;
    const int64_t n_items = fused ? a.n_sd : *a.n_live_in;
    const bool lds = a.lds_bins > 0;
    const int64_t pair0 = (int64_t)blockIdx.x * (THREADS * EPT / 2);

    uint64_t key[EPT];
    uint64_t xv[EPT];
    uint32_t bk[EPT];
    uint32_t rk[EPT];
    uint32_t sid[EPT];

#pragma unroll
    for (int k = 0; k < EPT / 2; ++k) {
        const int64_t p = pair0 + (int64_t)k * THREADS + tid;
        const int64_t i0 = 2 * p;
        uint32_t s[2];
        bool live[2];
        int32_t cell[2];
        uint64_t x[2] = {0, 0};
        if (fused) {
            s[0] = (uint32_t)i0;
            s[1] = (uint32_t)(i0 + 1);
            if (i0 + 1 < n_items) {
                const ulonglong2 xx = *reinterpret_cast<const ulonglong2 *>(a.xi + i0);
                x[0] = xx.x;
                x[1] = xx.y;
            } else if (i0 < n_items) {
                x[0] = a.xi[i0];
            }
            live[0] = x[0] > 0;
            live[1] = x[1] > 0;
        } else {
            live[0] = i0 < n_items;
            live[1] = i0 + 1 < n_items;
            s[0] = live[0] ? a.idx_in[i0] : 0;
            s[1] = live[1] ? a.idx_in[i0 + 1] : 0;
        }
        // cells
        int seg = 0;
        if (a.seg_off) {
            seg = find_seg(a.seg_off, a.n_cell, s[0]);
            cell[0] = cell[1] = seg;
            if (!fused)
                cell[1] = find_seg(a.seg_off, a.n_cell, s[1]);
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
        // shuffle keys
        uint64_t kk[2] = {0, 0};
        if (a.mode == MODE_CELLSORT) {
            kk[0] = (uint64_t)i0 << a.key_shift;
            kk[1] = (uint64_t)(i0 + 1) << a.key_shift;
        } else if (a.u01) {
#pragma unroll
            for (int e = 0; e < 2; ++e)
                kk[e] = live[e] ? uniform_to_key(a.u01[s[e]]) : 0;
        } else if (fused) {
            if (live[0] || live[1]) {
                uint32_t run = a.run;
                uint64_t lp = (uint64_t)p;
                if (a.seg_off) {
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
            key[j] = kk[e];
            xv[j] = x[e];
            sid[j] = s[e];
            bk[j] = NO_BUCKET;
            rk[j] = 0;
            if (live[e]) {
                const int h = a.cell_h[cell[e]];
                const uint32_t b = (uint32_t)a.cell_bucket_base[cell[e]] +
                                   (h ? (uint32_t)(kk[e] >> (53 - h)) : 0u);
                bk[j] = b;
                rk[j] = lds ? atomicAdd(&hist[b], 1u) : atomicAdd(&a.cursor[b], 1u);
            }
        }
    }
    __syncthreads();
    if (lds) {
        for (int b = tid; b < a.B; b += THREADS) {
            const uint32_t c = hist[b];
            if (c)
                hist[b] = atomicAdd(&a.cursor[b], c);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint32_t b = bk[j];
        if (b == NO_BUCKET)
            continue;
        const uint32_t pos = (lds ? hist[b] : 0u) + rk[j];
        const uint32_t base = a.slot_base[b];
        const uint32_t cap = a.slot_base[b + 1] - base;
        if (pos < cap) {
            const uint32_t slot = base + pos;
            a.rec_key[slot] = key[j];
            a.rec_s[slot] = sid[j];
            if (fused) {
                a.rec_xi[slot] = xv[j];
                a.rec_v[slot] = a.v[sid[j]];
            }
        } else {
            const uint32_t o = atomicAdd(a.ov_count, 1u);
            a.ov_key[o] = key[j];
            a.ov_s[o] = sid[j];
            a.ov_bucket[o] = b;
        }
    }

    // The last workgroup turns bucket counts into ranks and cell starts.
    __threadfence();
    __syncthreads();
    if (tid == 0)
        s_last = atomicAdd(a.ticket, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last)
        return;
    __threadfence();
    const int B = a.B;
    const int chunk = (B + THREADS - 1) / THREADS;
    const int lo = min(B, tid * chunk), hi = min(B, lo + chunk);
    uint32_t sum = 0;
    for (int b = lo; b < hi; ++b)
        sum += load_agent(&a.cursor[b]);
    uint32_t total;
    uint32_t run = block_exclusive_scan<THREADS>(sum, scan_scratch, &total);
    for (int b = lo; b < hi; ++b) {
        a.rank_off[b] = run;
        run += load_agent(&a.cursor[b]);
    }
    if (tid == 0) {
        a.rank_off[B] = total;
        *a.n_live_out = (int64_t)total;
        *a.ticket = 0;
    }
    __threadfence_block();
    __syncthreads();
    for (int c = tid; c <= a.n_cell; c += THREADS)
        a.cell_start[c] = a.rank_off[a.cell_bucket_base[c]];
}

// ------------------------------------------------------- pair evaluation
struct CellCtx {
    int32_t c;
    uint32_t cs, ce;
};

struct PairEnv {
    const uint64_t *seg_dummy;
};

// Evaluates one pair (eq. 3, gamma, eqs. 4-6) and writes back on collision.
template <class Args>
__device__ __forceinline__ void do_pair(const Args &a, uint32_t step, int32_t c,
                                        uint32_t cs, uint32_t ce, uint32_t r,
                                        uint32_t sa, uint64_t xa, double va,
                                        uint32_t sb_, uint64_t xb, double vb,
                                        Stats &st)
{
    double dvc;
    KernelDesc kd;
    uint32_t run;
    uint32_t gbase = 0;
    if (a.seg_run) {
        dvc = a.seg_dv[c];
        kd = a.kernels[a.seg_kernel[c]];
        run = (uint32_t)a.seg_run[c];
        gbase = a.seg_off[c] >> 1;
    } else {
        dvc = a.dv_cell ? a.dv_cell[c] : a.dv;
        kd = a.kern;
        run = a.run;
    }
    const uint64_t n_c = (uint64_t)(ce - cs);
    const double norm = (a.dt / dvc) * (double)pair_scale(n_c);
    const double ak = kernel_value(kd, va, vb);
    const uint64_t xm = xa > xb ? xa : xb;
    const double p = (ak * (double)xm) * norm;
    const uint32_t q = (r - (a.slot_cell_local ? cs : 0u)) >> 1;
    const double phi = word_to_uniform(philox_word(a.seed, run, step, SDM_STREAM_GAMMA, q));
    const double gamma = ceil(p - phi);
    if (a.gamma_out)
        a.gamma_out[gbase + q] = gamma;
    const Collision col = collide(xa, xb, gamma, st);
    if (col.g)
        apply_collision(col, sa, sb_, a.xi, a.attr, a.n_attr, a.stride);
}

// Output phase shared by the LDS and the global-memory paths: idx, pairs,
// seam records.  Get provides s/xi/v of the element at local position f.
template <int THREADS, class Get>
__device__ void group_outputs(const GroupArgs &a, int g, int b0, int nb, uint32_t tot,
                              uint32_t rank0, const uint32_t *t_off, const Get &get,
                              uint32_t *red, uint32_t *s_state)
{
    const int tid = threadIdx.x;
    for (uint32_t f = tid; f < tot; f += THREADS)
        a.idx_out[rank0 + f] = get.s(f);
    if (a.mode != MODE_FUSED)
        return;
    const uint32_t step = step_of(a.step, a.step_dev);
    Stats st{0, 0, 0, 0, 0};
    if (tid == 0)
        *s_state = 0;
    __syncthreads();
    int bl = 0;
    for (uint32_t f = tid; f < tot; f += THREADS) {
        // bucket of f (t_off ascending, t_off[nb] = tot)
        int lo = 0, hi = nb;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (t_off[mid] <= f)
                lo = mid;
            else
                hi = mid;
        }
        bl = lo;
        const int32_t c = a.bucket_cell[b0 + bl];
        const uint32_t cs = a.cell_start[c], ce = a.cell_start[c + 1];
        const uint32_t r = rank0 + f;
        const uint32_t ic = r - cs;
        const bool opener = ((ic & 1u) == 0u) && (r + 1 < ce);
        if (opener) {
            if (f + 1 < tot) {
                do_pair(a, step, c, cs, ce, r, get.s(f), get.xi(f), get.v(f),
                        get.s(f + 1), get.xi(f + 1), get.v(f + 1), st);
            } else {
                SeamRec rec;
                rec.xi = get.xi(f);
                rec.v = get.v(f);
                rec.s = get.s(f);
                rec.rank = r;
                rec.cell = c;
                rec.pad = 0;
                a.seam_open[g] = rec;
                atomicOr(s_state, 1u);
            }
        } else if (f == 0 && (ic & 1u)) {
            SeamRec rec;
            rec.xi = get.xi(f);
            rec.v = get.v(f);
            rec.s = get.s(f);
            rec.rank = r;
            rec.cell = c;
            rec.pad = 0;
            a.seam_close[g] = rec;
            atomicOr(s_state, 2u);
        }
    }
    flush_stats<THREADS>(st, a.counters, red);
    if (tid == 0) {
        a.seam_state[g] = *s_state;
        a.group_tot[g] = tot;
    }
}

struct LdsGet {
    const uint32_t *SF;
    const uint64_t *XF;
    const double *VF;
    __device__ uint32_t s(uint32_t f) const { return SF[f]; }
    __device__ uint64_t xi(uint32_t f) const { return XF[f]; }
    __device__ double v(uint32_t f) const { return VF[f]; }
};

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

// --------------------------------------------------------------- k_group
template <int THREADS, int EPT>
__global__ __launch_bounds__(THREADS) void k_group(GroupArgs a)
{
    constexpr int CAP = THREADS * EPT;
    __shared__ uint32_t t_off[MAXB + 1];
    __shared__ uint32_t t_cnt[MAXB];
    __shared__ uint32_t t_subbase[MAXB + 1];
    __shared__ uint32_t t_shift[MAXB];
    __shared__ uint32_t t_mask[MAXB];
    __shared__ uint32_t sub_hist[NSUB + 1];
    __shared__ uint32_t red[5 * (THREADS / 64) + 8];
    __shared__ uint32_t s_misc[4];
    __shared__ __align__(16) unsigned char pool[CAP * 20];

    const int tid = threadIdx.x;
    const int g = blockIdx.x;
    const int b0 = a.group_first[g], b1 = a.group_first[g + 1];
    const int nb = b1 - b0;
    for (int i = tid; i < nb; i += THREADS) {
        const int b = b0 + i;
        t_cnt[i] = a.cursor[b];
        const int h = a.cell_h[a.bucket_cell[b]];
        const int u = a.sub_bits[b];
        t_shift[i] = (uint32_t)(53 - h - u);
        t_mask[i] = (1u << u) - 1u;
        t_subbase[i] = 1u << u;  // count, scanned below
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t off = 0, sub = 0, ovf = 0;
        for (int i = 0; i < nb; ++i) {
            const uint32_t c = t_cnt[i];
            const uint32_t cap = a.slot_base[b0 + i + 1] - a.slot_base[b0 + i];
            if (c > cap)
                ovf = 1;
            t_off[i] = off;
            off += c;
            const uint32_t ns = t_subbase[i];
            t_subbase[i] = sub;
            sub += ns;
        }
        t_off[nb] = off;
        t_subbase[nb] = sub;
        s_misc[0] = off;
        s_misc[1] = ovf;
    }
    __syncthreads();
    const uint32_t tot = s_misc[0];
    const bool ovf = s_misc[1] != 0;
    const uint32_t rank0 = a.rank_off[b0];
    // reset the bucket cursors for the next launch (counts are in LDS)
    for (int i = tid; i < nb; i += THREADS)
        a.cursor[b0 + i] = 0;
    const uint32_t cap_here = a.group_cap >= 0 ? (uint32_t)min(a.group_cap, CAP) : (uint32_t)CAP;
    const bool fused = a.mode == MODE_FUSED;

    if (tot <= cap_here && !ovf) {
        // ------------------------------------------------ LDS path
        uint64_t *K1 = reinterpret_cast<uint64_t *>(pool);
        uint32_t *S1 = reinterpret_cast<uint32_t *>(pool + 8 * CAP);
        uint16_t *O1 = reinterpret_cast<uint16_t *>(pool + 12 * CAP);
        uint16_t *SB1 = reinterpret_cast<uint16_t *>(pool + 14 * CAP);
        uint16_t *FP = reinterpret_cast<uint16_t *>(pool + 16 * CAP);
        const uint32_t nsub = t_subbase[nb];
        for (uint32_t i = tid; i <= nsub; i += THREADS)
            sub_hist[i] = 0;
        __syncthreads();
        uint64_t key[EPT], xv[EPT];
        double vv[EPT];
        uint32_t sid[EPT], sbk[EPT], lrk[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const uint32_t li = (uint32_t)(e * THREADS + tid);
            sbk[e] = NO_BUCKET;
            if (li < tot) {
                int lo = 0, hi = nb;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (t_off[mid] <= li)
                        lo = mid;
                    else
                        hi = mid;
                }
                const uint32_t slot = a.slot_base[b0 + lo] + (li - t_off[lo]);
                key[e] = a.rec_key[slot];
                sid[e] = a.rec_s[slot];
                if (fused) {
                    xv[e] = a.rec_xi[slot];
                    vv[e] = a.rec_v[slot];
                } else {
                    xv[e] = 0;
                    vv[e] = 0.0;
                }
                const uint32_t sub = (uint32_t)(key[e] >> t_shift[lo]) & t_mask[lo];
                sbk[e] = t_subbase[lo] + sub;
                lrk[e] = atomicAdd(&sub_hist[sbk[e]], 1u);
            }
        }
        __syncthreads();
        // exclusive scan of the sub-bucket histogram (nsub <= NSUB)
        {
            constexpr int PER = (NSUB + THREADS - 1) / THREADS;
            uint32_t loc[PER];
            uint32_t sum = 0;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const uint32_t idx = tid * PER + i;
                loc[i] = idx < nsub ? sub_hist[idx] : 0u;
                sum += loc[i];
            }
            uint32_t total;
            uint32_t run = block_exclusive_scan<THREADS>(sum, red, &total);
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const uint32_t idx = tid * PER + i;
                if (idx < nsub)
                    sub_hist[idx] = run;
                run += loc[i];
            }
            if (tid == 0)
                sub_hist[nsub] = total;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if (sbk[e] != NO_BUCKET) {
                const uint32_t pos = sub_hist[sbk[e]] + lrk[e];
                K1[pos] = key[e];
                S1[pos] = sid[e];
                O1[pos] = (uint16_t)(e * THREADS + tid);
                SB1[pos] = (uint16_t)sbk[e];
            }
        }
        __syncthreads();
        // exact rank inside each sub-bucket by (key, s)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const uint32_t pos = (uint32_t)(e * THREADS + tid);
            if (pos < tot) {
                const uint64_t k = K1[pos];
                const uint32_t s = S1[pos];
                const uint32_t b = SB1[pos];
                const uint32_t lo = sub_hist[b], hi = sub_hist[b + 1];
                uint32_t r = 0;
                for (uint32_t q = lo; q < hi; ++q) {
                    const uint64_t kq = K1[q];
                    r += (kq < k) || (kq == k && S1[q] < s);
                }
                FP[O1[pos]] = (uint16_t)(lo + r);
            }
        }
        __syncthreads();
        uint32_t fp[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            if (sbk[e] != NO_BUCKET)
                fp[e] = FP[e * THREADS + tid];
        __syncthreads();
        uint64_t *XF = reinterpret_cast<uint64_t *>(pool);
        double *VF = reinterpret_cast<double *>(pool + 8 * CAP);
        uint32_t *SF = reinterpret_cast<uint32_t *>(pool + 16 * CAP);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if (sbk[e] != NO_BUCKET) {
                XF[fp[e]] = xv[e];
                VF[fp[e]] = vv[e];
                SF[fp[e]] = sid[e];
            }
        }
        __syncthreads();
        LdsGet get{SF, XF, VF};
        group_outputs<THREADS>(a, g, b0, nb, tot, rank0, t_off, get, red, &s_misc[2]);
        return;
    }

    // ---------------------------------------------------- global path
    // Gather the group's records (bucket regions + overflow list) into
    // scratch at [2 rank0, 2 rank0 + P), P = next power of two >= tot, and
    // sort them there by (bucket, key, s) with a bitonic network.  The
    // ranges of consecutive groups are disjoint because P <= 2 tot.
    if (tot == 0) {
        GlobalGet none{a.ss, nullptr, nullptr};
        group_outputs<THREADS>(a, g, b0, nb, 0, rank0, t_off, none, red, &s_misc[2]);
        return;
    }
    const uint32_t base2 = 2u * rank0;
    uint32_t P = 1;
    while (P < tot)
        P <<= 1;
    if (tid == 0)
        s_misc[3] = 0;
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        const uint32_t cap = a.slot_base[b0 + i + 1] - a.slot_base[b0 + i];
        const uint32_t m = min(t_cnt[i], cap);
        for (uint32_t j = tid; j < m; j += THREADS) {
            const uint32_t slot = a.slot_base[b0 + i] + j;
            const uint32_t pos = atomicAdd(&s_misc[3], 1u);
            a.sk[base2 + pos] = a.rec_key[slot];
            a.ss[base2 + pos] = a.rec_s[slot];
            a.sb[base2 + pos] = (uint32_t)i;
        }
    }
    if (ovf) {
        const uint32_t n_ov = *a.ov_count;
        for (uint32_t i = tid; i < n_ov; i += THREADS) {
            const uint32_t b = a.ov_bucket[i];
            if (b >= (uint32_t)b0 && b < (uint32_t)b1) {
                const uint32_t pos = atomicAdd(&s_misc[3], 1u);
                a.sk[base2 + pos] = a.ov_key[i];
                a.ss[base2 + pos] = a.ov_s[i];
                a.sb[base2 + pos] = b - (uint32_t)b0;
            }
        }
    }
    __syncthreads();
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
    group_outputs<THREADS>(a, g, b0, nb, tot, rank0, t_off, get, red, &s_misc[2]);
}

// --------------------------------------------------------------- k_seams
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_seams(SeamArgs a)
{
    __shared__ uint32_t red[5 * (THREADS / 64) + 8];
    __shared__ int s_last;
    const int g = blockIdx.x * THREADS + threadIdx.x;
    const uint32_t step = step_of(a.step, a.step_dev);
    Stats st{0, 0, 0, 0, 0};
    if (a.mode == MODE_FUSED && g < a.G && (a.seam_state[g] & 1u)) {
        const SeamRec op = a.seam_open[g];
        int g2 = g + 1;
        while (g2 < a.G && a.group_tot[g2] == 0)
            ++g2;
        if (g2 < a.G) {
            const SeamRec cl = a.seam_close[g2];
            const uint32_t cs = a.cell_start[op.cell], ce = a.cell_start[op.cell + 1];
            do_pair(a, step, op.cell, cs, ce, op.rank, op.s, op.xi, op.v, cl.s, cl.xi,
                    cl.v, st);
        }
    }
    if (a.mode == MODE_FUSED)
        flush_stats<THREADS>(st, a.counters, red);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *a.ov_count = 0;
    // the last workgroup advances the device step counter
    if (a.step_advance) {
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0)
            s_last = atomicAdd(a.ticket, 1u) == gridDim.x - 1;
        __syncthreads();
        if (s_last && threadIdx.x == 0) {
            *a.step_advance = *a.step_advance + 1u;
            *a.ticket = 0;
        }
    }
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

// Describes one cell (or run) for plan building.
struct CellPlanIn {
    double expected;  // expected live SDs
};

static Plan *build_plan(sdm_ctx *ctx, int mode, int64_t n_items,
                        const std::vector<double> &expected, bool batched)
{
    Plan *p = new Plan();
    try {
        const int32_t C = (int32_t)expected.size();
        p->mode = mode;
        p->n_items = n_items;
        p->n_cell = C;
        std::vector<int32_t> cell_h(C), cell_bb(C + 1);
        std::vector<int32_t> bucket_cell;
        std::vector<uint32_t> slot_base;
        std::vector<uint8_t> sub_bits;
        std::vector<double> bucket_exp;
        uint64_t slots = 0;
        int32_t B = 0;
        for (int32_t c = 0; c < C; ++c) {
            const double m = std::max(expected[c], 1.0);
            int h = 0;
            if (mode != MODE_CELLSORT || true) {
                while (m / std::ldexp(1.0, h) > BUCKET_TARGET && h < 24)
                    ++h;
            }
            cell_h[c] = h;
            cell_bb[c] = B;
            const double e = m / std::ldexp(1.0, h);
            uint32_t cap;
            if (ctx->dbg_bucket_cap > 0)
                cap = (uint32_t)ctx->dbg_bucket_cap;
            else
                cap = (uint32_t)(std::ceil((e + 10.0 * std::sqrt(e) + 64.0) / 64.0) * 64.0);
            int u = 0;
            while (e / std::ldexp(1.0, u + 1) >= 4.0 && u < 10)
                ++u;
            if (u > 53 - h)
                u = 53 - h;
            for (int i = 0; i < (1 << h); ++i) {
                bucket_cell.push_back(c);
                slot_base.push_back((uint32_t)slots);
                sub_bits.push_back((uint8_t)u);
                bucket_exp.push_back(e);
                slots += cap;
                ++B;
            }
        }
        cell_bb[C] = B;
        slot_base.push_back((uint32_t)slots);
        if (slots >= 0xFFFFFFF0ull)
            throw HipError{hipErrorOutOfMemory, "plan too large"};
        // groups: consecutive buckets with expected total <= GROUP_TARGET
        std::vector<int32_t> group_first;
        {
            int32_t b = 0;
            while (b < B) {
                group_first.push_back(b);
                double acc = 0;
                int nsub = 0, n = 0;
                while (b < B) {
                    const int ns = 1 << sub_bits[b];
                    if (n > 0 && (acc + bucket_exp[b] > GROUP_TARGET || n + 1 > MAXB ||
                                  nsub + ns > NSUB))
                        break;
                    acc += bucket_exp[b];
                    nsub += ns;
                    ++n;
                    ++b;
                }
            }
            group_first.push_back(B);
        }
        p->B = B;
        p->G = (int32_t)group_first.size() - 1;
        p->S = (uint32_t)slots;
        p->lds_bins = B <= LDS_BINS_MAX ? B : 0;
        p->cell_h = upload(p, cell_h);
        p->cell_bucket_base = upload(p, cell_bb);
        p->bucket_cell = upload(p, bucket_cell);
        p->slot_base = upload(p, slot_base);
        p->sub_bits = upload(p, sub_bits);
        p->group_first = upload(p, group_first);
        const bool fused = mode == MODE_FUSED;
        p->cursor = (uint32_t *)dalloc(p, 4ull * B);
        p->rank_off = (uint32_t *)dalloc(p, 4ull * (B + 1));
        p->cell_start_ws = (uint32_t *)dalloc(p, 4ull * (C + 1));
        p->n_live_ws = (int64_t *)dalloc(p, 8);
        p->ticket = (uint32_t *)dalloc(p, 16);
        p->rec_key = (uint64_t *)dalloc(p, 8ull * slots);
        p->rec_s = (uint32_t *)dalloc(p, 4ull * slots);
        if (fused) {
            p->rec_xi = (uint64_t *)dalloc(p, 8ull * slots);
            p->rec_v = (double *)dalloc(p, 8ull * slots);
        }
        p->ov_count = (uint32_t *)dalloc(p, 16);
        p->ov_key = (uint64_t *)dalloc(p, 8ull * n_items + 8);
        p->ov_s = (uint32_t *)dalloc(p, 4ull * n_items + 8);
        p->ov_bucket = (uint32_t *)dalloc(p, 4ull * n_items + 8);
        p->sk = (uint64_t *)dalloc(p, 16ull * n_items + 64);
        p->ss = (uint32_t *)dalloc(p, 8ull * n_items + 64);
        p->sb = (uint32_t *)dalloc(p, 8ull * n_items + 64);
        p->seam_open = (SeamRec *)dalloc(p, sizeof(SeamRec) * p->G);
        p->seam_close = (SeamRec *)dalloc(p, sizeof(SeamRec) * p->G);
        p->seam_state = (uint32_t *)dalloc(p, 4ull * p->G);
        p->group_tot = (uint32_t *)dalloc(p, 4ull * p->G);
        SDM_HIP(hipMemset(p->cursor, 0, 4ull * B));
        SDM_HIP(hipMemset(p->ticket, 0, 16));
        SDM_HIP(hipMemset(p->ov_count, 0, 16));
        SDM_HIP(hipMemset(p->seam_state, 0, 4ull * p->G));
        SDM_HIP(hipMemset(p->group_tot, 0, 4ull * p->G));
        SDM_HIP(hipDeviceSynchronize());
        (void)batched;
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
    Plan *p = build_plan(ctx, mode, n_items, exp, false);
    ctx->plans[key] = p;
    return p;
}

static void set_kernel_attributes()
{
    static bool done = false;
    if (done)
        return;
    SDM_HIP(hipFuncSetAttribute((const void *)k_scatter<SCATTER_THREADS, SCATTER_EPT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                LDS_BINS_MAX * 4 + 1024));
    done = true;
}

void engine_run(sdm_ctx *ctx, Plan *p, const StepInputs &in, hipStream_t stream)
{
    set_kernel_attributes();
    const bool fused = p->mode == MODE_FUSED;
    uint32_t *cell_start = in.cell_start ? in.cell_start : p->cell_start_ws;
    int64_t *n_live_out = in.n_live_out ? in.n_live_out : p->n_live_ws;

    ScatterArgs sa{};
    sa.mode = p->mode;
    sa.n_sd = in.n_sd;
    sa.n_live_in = in.n_live_in;
    sa.idx_in = in.idx_in;
    sa.xi = in.xi;
    sa.v = in.attr;
    sa.cell_id = in.cell_id;
    sa.n_cell = p->n_cell;
    sa.u01 = in.u01;
    sa.seed = in.seed;
    sa.run = in.run;
    sa.step = in.step;
    sa.step_dev = in.step_dev;
    sa.key_shift = 53 - std::max(1, ceil_log2_u64((uint64_t)std::max<int64_t>(p->n_items, 2)));
    sa.cell_h = p->cell_h;
    sa.cell_bucket_base = p->cell_bucket_base;
    sa.slot_base = p->slot_base;
    sa.B = p->B;
    sa.lds_bins = p->lds_bins;
    sa.seg_off = p->seg_off;
    sa.seg_run = p->seg_run;
    sa.cursor = p->cursor;
    sa.rec_key = p->rec_key;
    sa.rec_s = p->rec_s;
    sa.rec_xi = p->rec_xi;
    sa.rec_v = p->rec_v;
    sa.ov_count = p->ov_count;
    sa.ov_key = p->ov_key;
    sa.ov_s = p->ov_s;
    sa.ov_bucket = p->ov_bucket;
    sa.rank_off = p->rank_off;
    sa.cell_start = cell_start;
    sa.n_live_out = n_live_out;
    sa.ticket = p->ticket;
    sa.err = ctx->err_dev;
    auto mark = [&](int i) {
        if (in.events[i])
            SDM_HIP(hipEventRecord(in.events[i], stream));
    };
    const int64_t items = fused ? in.n_sd : p->n_items;
    const int64_t per_block = (int64_t)SCATTER_THREADS * SCATTER_EPT;
    const int grid1 = (int)std::max<int64_t>(1, (items + per_block - 1) / per_block);
    mark(0);
    hipLaunchKernelGGL((k_scatter<SCATTER_THREADS, SCATTER_EPT>), dim3(grid1),
                       dim3(SCATTER_THREADS), (size_t)p->lds_bins * 4, stream, sa);
    SDM_HIP(hipGetLastError());

    GroupArgs ga{};
    ga.mode = p->mode;
    ga.group_first = p->group_first;
    ga.bucket_cell = p->bucket_cell;
    ga.slot_base = p->slot_base;
    ga.sub_bits = p->sub_bits;
    ga.cell_h = p->cell_h;
    ga.cursor = p->cursor;
    ga.rank_off = p->rank_off;
    ga.cell_start = cell_start;
    ga.rec_key = p->rec_key;
    ga.rec_s = p->rec_s;
    ga.rec_xi = p->rec_xi;
    ga.rec_v = p->rec_v;
    ga.ov_count = p->ov_count;
    ga.ov_key = p->ov_key;
    ga.ov_s = p->ov_s;
    ga.ov_bucket = p->ov_bucket;
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
    mark(1);
    hipLaunchKernelGGL((k_group<GROUP_THREADS, GROUP_EPT>), dim3(p->G), dim3(GROUP_THREADS), 0,
                       stream, ga);
    SDM_HIP(hipGetLastError());

    SeamArgs ta{};
    ta.mode = p->mode;
    ta.G = p->G;
    ta.seam_open = p->seam_open;
    ta.seam_close = p->seam_close;
    ta.seam_state = p->seam_state;
    ta.group_tot = p->group_tot;
    ta.cell_start = cell_start;
    ta.xi = in.xi;
    ta.attr = in.attr;
    ta.n_attr = in.n_attr;
    ta.stride = in.stride;
    ta.dt = in.dt;
    ta.dv_cell = in.dv_cell;
    ta.dv = in.dv;
    ta.kern = in.kern;
    ta.seg_off = p->seg_off;
    ta.seg_run = p->seg_run;
    ta.seg_kernel = p->seg_kernel;
    ta.seg_dv = p->seg_dv;
    ta.kernels = p->kernels;
    ta.seed = in.seed;
    ta.run = in.run;
    ta.step = in.step;
    ta.step_dev = in.step_dev;
    ta.slot_cell_local = in.slot_cell_local ? 1 : 0;
    ta.counters = in.counters;
    ta.gamma_out = in.gamma_out;
    ta.ov_count = p->ov_count;
    ta.ticket = p->ticket + 1;
    ta.step_advance = in.step_advance;
    constexpr int ST = 256;
    const int grid3 = std::max(1, (p->G + ST - 1) / ST);
    mark(2);
    hipLaunchKernelGGL((k_seams<ST>), dim3(grid3), dim3(ST), 0, stream, ta);
    SDM_HIP(hipGetLastError());
    mark(3);
    (void)fused;
}

}  // namespace sdm
