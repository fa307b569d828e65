/*
 * sdm_oracle.c -- plain single-threaded C99 reference of the Super-Droplet
 * Method coagulation step (arXiv:2101.06318).  TEST INFRASTRUCTURE ONLY: see
 * sdm_oracle.h.  Each function names the passage of the paper it follows.
 *
 * Floating point: binary64, round-to-nearest-even, every operation written
 * out in the order evaluated; built with -ffp-contract=off (no fused
 * multiply-add) and without fast-math.
 */
#include "sdm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon, Moraes, Dror & Shaw,      */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): per round the    */
/* two multipliers act on counter words 0 and 2; the high halves are mixed */
/* with the other two counter words and the round key; the key is bumped   */
/* by the two Weyl constants between rounds.                               */
/* ------------------------------------------------------------------------ */
void sdmo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                        uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint64_t sdmo_word(uint64_t seed, uint32_t run, uint32_t step,
                   uint32_t stream, uint64_t e)
{
    uint32_t ctr[4], key[2], out[4];
    ctr[0] = (uint32_t)(e >> 1);
    ctr[1] = step;
    ctr[2] = stream;
    ctr[3] = run;
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    sdmo_philox4x32_10(ctr, key, out);
    if (e & 1u)
        return ((uint64_t)out[2] << 32) | (uint64_t)out[3];
    return ((uint64_t)out[0] << 32) | (uint64_t)out[1];
}

/* 2^-53 as an exact binary64 constant. */
#define SDMO_TWO_M53 (1.0 / 9007199254740992.0)

double sdmo_uniform(uint64_t seed, uint32_t run, uint32_t step,
                    uint32_t stream, uint64_t e)
{
    uint64_t w = sdmo_word(seed, run, step, stream, e);
    return (double)(w >> 11) * SDMO_TWO_M53;
}

/* urand: the paper's Step 1 and Step 3 draw u01 ~ U[0,1). */
void sdmo_urand(double *u01, int64_t n, uint64_t seed, uint32_t run,
                uint32_t step, uint32_t stream)
{
    int64_t e;
    for (e = 0; e < n; ++e)
        u01[e] = sdmo_uniform(seed, run, step, stream, (uint64_t)e);
}

static int32_t cell_of(const int32_t *cell_id, uint32_t s)
{
    return cell_id ? cell_id[s] : 0;
}

/* ------------------------------------------------------------------------ */
/* Step 0 (Sec. 3.2: super-droplets of zero multiplicity are dropped from   */
/* the Index at the start of each timestep).  Stable filter.                */
/* ------------------------------------------------------------------------ */
int64_t sdmo_remove_if_equal_0(uint32_t *idx, int64_t n_live, const uint64_t *xi)
{
    int64_t i, m = 0;
    for (i = 0; i < n_live; ++i)
        if (xi[idx[i]] > 0)
            idx[m++] = idx[i];
    return m;
}

/* ------------------------------------------------------------------------ */
/* Step 1.  The Index is sorted with the cell id as key (Sec. 3.1); the     */
/* shuffle is a sort with random keys (Sec. 3.2, GPU strategy).             */
/* ------------------------------------------------------------------------ */
static int fill_cell_start(uint32_t *cell_start, const uint32_t *idx,
                           int64_t n_live, const int32_t *cell_id,
                           int32_t n_cell)
{
    int64_t i;
    int32_t c;
    for (c = 0; c <= n_cell; ++c)
        cell_start[c] = 0;
    for (i = 0; i < n_live; ++i) {
        int32_t ci = cell_of(cell_id, idx[i]);
        if (ci < 0 || ci >= n_cell)
            return -1;
        cell_start[ci + 1] += 1;
    }
    for (c = 0; c < n_cell; ++c)
        cell_start[c + 1] += cell_start[c];
    return 0;
}

int sdmo_cell_sort(uint32_t *cell_start, uint32_t *idx, int64_t n_live,
                   const int32_t *cell_id, int32_t n_cell)
{
    uint32_t *pos, *out;
    int64_t i;
    int32_t c;
    if (fill_cell_start(cell_start, idx, n_live, cell_id, n_cell))
        return -1;
    pos = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n_cell + 1));
    out = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n_live + 1));
    for (c = 0; c <= n_cell; ++c)
        pos[c] = cell_start[c];
    for (i = 0; i < n_live; ++i) {
        int32_t ci = cell_of(cell_id, idx[i]);
        out[pos[ci]++] = idx[i];
    }
    memcpy(idx, out, sizeof(uint32_t) * (size_t)n_live);
    free(pos);
    free(out);
    return 0;
}

/* Uniform integer in [0, m) from the 53-bit word of element e. */
static uint64_t draw_below(uint64_t seed, uint32_t run, uint32_t step, uint32_t stream,
                           uint64_t e, uint64_t m)
{
    uint64_t w = sdmo_word(seed, run, step, stream, e) >> 11;
    return (uint64_t)(((unsigned __int128)w * m) >> 53);
}

static void swap_u32(uint32_t *a, uint32_t *b)
{
    uint32_t t = *a;
    *a = *b;
    *b = t;
}

/* Fisher-Yates on positions [s, e) of idx, draws keyed by position. */
static void fisher_yates(uint32_t *idx, int64_t s, int64_t e, uint64_t seed, uint32_t run,
                         uint32_t step)
{
    int64_t i;
    for (i = e - 1; i > s; --i) {
        uint64_t k = draw_below(seed, run, step, SDMO_STREAM_FY, (uint64_t)i,
                                (uint64_t)(i - s + 1));
        swap_u32(&idx[i], &idx[s + (int64_t)k]);
    }
}

int sdmo_shuffle_fisher_yates(uint32_t *cell_start, uint32_t *idx, int64_t n_live,
                              const int32_t *cell_id, int32_t n_cell, uint64_t seed,
                              uint32_t run, uint32_t step)
{
    int32_t c;
    if (sdmo_cell_sort(cell_start, idx, n_live, cell_id, n_cell))
        return -1;
    for (c = 0; c < n_cell; ++c)
        fisher_yates(idx, cell_start[c], cell_start[c + 1], seed, run, step);
    return 0;
}

/* One merge of MergeShuffle at level d: [s, m) and [m, e) are shuffled. */
static void merge_shuffled(uint32_t *idx, int64_t s, int64_t m, int64_t e, int d,
                           uint64_t seed, uint32_t run, uint32_t step)
{
    int64_t i = s, j = m;
    for (;;) {
        uint64_t coin = sdmo_word(seed, run, step, SDMO_STREAM_MERGE + 2 * d, (uint64_t)i) >> 63;
        if (coin == 0) {
            if (i == j)
                break;
        } else {
            if (j == e)
                break;
            swap_u32(&idx[i], &idx[j]);
            ++j;
        }
        ++i;
    }
    for (; i < e; ++i) {
        uint64_t k = draw_below(seed, run, step, SDMO_STREAM_MERGE + 2 * d + 1, (uint64_t)i,
                                (uint64_t)(i - s + 1));
        swap_u32(&idx[i], &idx[s + (int64_t)k]);
    }
}

int sdmo_shuffle_merge(uint32_t *cell_start, uint32_t *idx, int64_t n_live,
                       const int32_t *cell_id, int32_t n_cell, uint64_t seed, uint32_t run,
                       uint32_t step)
{
    int32_t c;
    if (sdmo_cell_sort(cell_start, idx, n_live, cell_id, n_cell))
        return -1;
    for (c = 0; c < n_cell; ++c) {
        int64_t cs = cell_start[c], ce = cell_start[c + 1], s, w;
        int d;
        for (s = cs; s < ce; s += 16)
            fisher_yates(idx, s, s + 16 < ce ? s + 16 : ce, seed, run, step);
        for (d = 1, w = 16; cs + w < ce; ++d, w *= 2)
            for (s = cs; s + w < ce; s += 2 * w)
                merge_shuffled(idx, s, s + w, s + 2 * w < ce ? s + 2 * w : ce, d, seed, run,
                               step);
    }
    return 0;
}

typedef struct {
    int32_t  cell;
    uint32_t s;
    uint64_t key;
} sort_item;

static int cmp_item(const void *a, const void *b)
{
    const sort_item *x = (const sort_item *)a, *y = (const sort_item *)b;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    return 0;
}

int sdmo_shuffle_per_cell(uint32_t *cell_start, uint32_t *idx, int64_t n_live,
                          const int32_t *cell_id, int32_t n_cell,
                          const double *u01_by_sd)
{
    sort_item *it;
    int64_t i;
    if (fill_cell_start(cell_start, idx, n_live, cell_id, n_cell))
        return -1;
    it = (sort_item *)malloc(sizeof(sort_item) * (size_t)(n_live + 1));
    for (i = 0; i < n_live; ++i) {
        uint32_t s = idx[i];
        it[i].cell = cell_of(cell_id, s);
        it[i].s = s;
        /* u in [0,1) scaled by 2^53 exactly; the key is its integer part */
        it[i].key = (uint64_t)(u01_by_sd[s] * 9007199254740992.0);
    }
    qsort(it, (size_t)n_live, sizeof(sort_item), cmp_item);
    for (i = 0; i < n_live; ++i)
        idx[i] = it[i].s;
    free(it);
    return 0;
}

/* flag_pairs: the pair-flag predicate of the GPU listing (Fig. 3). */
void sdmo_flag_pairs(uint8_t *flag, const int32_t *cell_id,
                     const uint32_t *cell_start, const uint32_t *idx,
                     int64_t n_live)
{
    int64_t i;
    for (i = 0; i < n_live; ++i) {
        int32_t c = cell_of(cell_id, idx[i]);
        int f = 0;
        if (i + 1 < n_live && cell_of(cell_id, idx[i + 1]) == c &&
            ((i - (int64_t)cell_start[c]) % 2) == 0)
            f = 1;
        flag[i] = (uint8_t)f;
    }
}

/* ------------------------------------------------------------------------ */
/* Coalescence kernels a(v1, v2).  Golovin (additive) b*(v1+v2) is the one  */
/* of the paper's validation case (Sec. 4); constant and multiplicative are */
/* the other analytically solvable kernels it lists (Sec. 2.1).  The        */
/* geometric (gravitational) kernel is pi (r1+r2)^2 |w1-w2| with a          */
/* three-regime power-law terminal velocity; the paper only names it.       */
/* ------------------------------------------------------------------------ */
#define SDMO_PI 3.141592653589793

double sdmo_cbrt(double x)
{
    int e, q, it;
    double y;
    if (x == 0.0)
        return 0.0;
    (void)frexp(x, &e); /* x = m * 2^e, m in [0.5, 1) */
    q = e / 3;
    if (e % 3 < 0)
        q -= 1; /* floor division */
    y = ldexp(1.0, q);
    for (it = 0; it < 8; ++it)
        y = (2.0 * y + x / (y * y)) / 3.0; /* Newton step for y^3 = x */
    return y;
}

/* Terminal velocity [m/s] of a drop of radius r [m]: the textbook
 * three-regime power law, k1 r^2 (Stokes), k2 r, then k3 sqrt(r), with
 * k1 = 1.19e8 1/(m s), k2 = 8e3 1/s, k3 = 201 m^0.5/s.  The paper names the
 * gravitational kernel's terminal velocity only as a parametric form
 * (Sec. 4); the reading here switches law where the adjacent laws meet,
 * r = k2/k1 (67.2 um) and r = (k3/k2)^2 (631 um), so that w(r) is
 * continuous and increasing. */
#define SDMO_VT_K1 1.19e8
#define SDMO_VT_K2 8.0e3
#define SDMO_VT_K3 201.0

double sdmo_terminal_velocity(double r)
{
    const double r12 = SDMO_VT_K2 / SDMO_VT_K1;
    const double r23 = (SDMO_VT_K3 / SDMO_VT_K2) * (SDMO_VT_K3 / SDMO_VT_K2);
    if (r < r12)
        return SDMO_VT_K1 * (r * r);
    if (r < r23)
        return SDMO_VT_K2 * r;
    return SDMO_VT_K3 * sqrt(r);
}

/* Cell of v in a tabulated kernel: the IEEE-754 bit pattern of v, as an
 * unsigned 64-bit integer, shifted right by 52 - m, minus lo, clamped to
 * [0, n - 1]. */
static int64_t sdmo_table_cell(double v, int64_t lo, int64_t n, int m)
{
    uint64_t bits;
    int64_t c;
    memcpy(&bits, &v, sizeof bits);
    c = (int64_t)(bits >> (52 - m)) - lo;
    if (c < 0)
        return 0;
    if (c > n - 1)
        return n - 1;
    return c;
}

double sdmo_kernel_value(int32_t kernel_id, const double *kparams,
                         const double *table, double v1, double v2)
{
    switch (kernel_id) {
    case SDMO_KERNEL_GOLOVIN:
        return kparams[0] * (v1 + v2);
    case SDMO_KERNEL_GEOMETRIC: {
        double r1 = sdmo_cbrt((0.75 * v1) / SDMO_PI);
        double r2 = sdmo_cbrt((0.75 * v2) / SDMO_PI);
        double w1 = sdmo_terminal_velocity(r1);
        double w2 = sdmo_terminal_velocity(r2);
        double rs = r1 + r2;
        return ((SDMO_PI * (rs * rs)) * fabs(w1 - w2)) * kparams[0];
    }
    case SDMO_KERNEL_CONSTANT:
        return kparams[0];
    case SDMO_KERNEL_MULTIPLICATIVE:
        return kparams[0] * (v1 * v2);
    case SDMO_KERNEL_TABULATED: {
        int64_t lo = (int64_t)kparams[1], n = (int64_t)kparams[2];
        int m = (int)kparams[3];
        int64_t i1 = sdmo_table_cell(v1, lo, n, m), i2 = sdmo_table_cell(v2, lo, n, m);
        int64_t r = i1 < i2 ? i1 : i2, c = i1 < i2 ? i2 : i1;
        return kparams[0] * table[r * n + c];
    }
    default:
        return 0.0;
    }
}

/* Step 2: coalescence_kernel, times_max, normalize (eq. 3, one factor per */
/* routine in the order of the workflow figure).                           */
void sdmo_coalescence_kernel(double *pair_prob, const uint8_t *flag,
                             const double *volume, const uint32_t *idx,
                             int64_t n_live, int32_t kernel_id,
                             const double *kparams, const double *table)
{
    int64_t i;
    for (i = 0; i < n_live / 2; ++i)
        pair_prob[i] = 0.0;
    for (i = 0; i < n_live; ++i)
        if (flag[i])
            pair_prob[i / 2] = sdmo_kernel_value(kernel_id, kparams, table,
                                                 volume[idx[i]], volume[idx[i + 1]]);
}

void sdmo_times_max(double *pair_prob, const uint64_t *xi, const uint8_t *flag,
                    const uint32_t *idx, int64_t n_live)
{
    int64_t i;
    for (i = 0; i < n_live; ++i)
        if (flag[i]) {
            uint64_t a = xi[idx[i]], b = xi[idx[i + 1]];
            uint64_t m = a > b ? a : b;
            pair_prob[i / 2] = pair_prob[i / 2] * (double)m;
        }
}

uint64_t sdmo_pair_scale(uint64_t n)
{
    if (n < 2)
        return 0;
    return ((n * n - n) / 2) / (n / 2);
}

void sdmo_normalize(double *pair_prob, double dt, const double *dv_per_cell,
                    const int32_t *cell_id, const uint32_t *cell_start,
                    const uint8_t *flag, const uint32_t *idx, int64_t n_live)
{
    int64_t i;
    for (i = 0; i < n_live; ++i)
        if (flag[i]) {
            int32_t c = cell_of(cell_id, idx[i]);
            uint64_t n_c = (uint64_t)(cell_start[c + 1] - cell_start[c]);
            double norm = (dt / dv_per_cell[c]) * (double)sdmo_pair_scale(n_c);
            pair_prob[i / 2] = pair_prob[i / 2] * norm;
        }
}

/* Step 3: gamma = ceil(p - phi), phi ~ U[0,1) (Sec. 2.2, Step 3). */
void sdmo_compute_gamma(double *pair_prob, const double *u01_by_slot,
                        int64_t n_slot)
{
    int64_t q;
    for (q = 0; q < n_slot; ++q)
        pair_prob[q] = ceil(pair_prob[q] - u01_by_slot[q]);
}

/* Rate gamma as an unsigned count: NaN, negative and -0.0 read as 0; values
 * at or above 2^64 saturate. */
static uint64_t gamma_count(double g)
{
    if (!(g >= 1.0))
        return 0;
    if (g >= 18446744073709551616.0)
        return UINT64_MAX;
    return (uint64_t)g;
}

/* update_attributes (Step 3), eqs. (4)-(6), for every pair (a, b) opened at
 * a flagged position i.  Of the two SDs, j has the larger multiplicity and
 * k the smaller (on equal multiplicities j is the one at the earlier
 * position).  Eq. (4): the number of collision events is
 * gt = min(gamma, floor(xi_j / xi_k)).  With gt > 0:
 *   eq. (5), gt xi_k < xi_j:  xi_j <- xi_j - gt xi_k,  A_k <- A_k + gt A_j;
 *   eq. (6), gt xi_k = xi_j:  xi_j <- floor(xi_k / 2),
 *                             xi_k <- xi_k - floor(xi_k / 2),
 *                             A_j, A_k <- A_k + gt A_j.
 * xi_j and A_j are unchanged in eq. (5), and xi_k, which never changes in
 * eq. (5), is split in eq. (6).  Counters: pairs visited, pairs with gt > 0,
 * pairs with gt < gamma, SDs whose multiplicity became 0, pairs with
 * gamma >= 2. */
void sdmo_update_attributes(uint64_t *xi, double *attr, int32_t n_attr,
                            int64_t attr_stride, const double *gamma,
                            const uint8_t *flag, const uint32_t *idx,
                            int64_t n_live, uint64_t *counters)
{
    int64_t i;
    int32_t r;
    for (i = 0; i < n_live; ++i) {
        uint32_t a, b, j, k;
        uint64_t events, cap, gt;
        if (!flag[i])
            continue;
        a = idx[i];
        b = idx[i + 1];
        j = xi[a] >= xi[b] ? a : b;
        k = j == a ? b : a;
        counters[SDMO_CNT_PAIRS] += 1;
        if (xi[k] == 0)
            continue; /* an SD already removed: nothing to collide with */
        events = gamma_count(gamma[i / 2]);
        cap = xi[j] / xi[k]; /* floor(xi_j / xi_k), exact in integers */
        gt = events < cap ? events : cap; /* eq. (4) */
        if (events >= 2)
            counters[SDMO_CNT_GAMMA_GE2] += 1;
        if (gt < events)
            counters[SDMO_CNT_CAPPED] += 1;
        if (gt == 0)
            continue;
        counters[SDMO_CNT_COLLISIONS] += 1;
        if (gt * xi[k] < xi[j]) {
            /* eq. (5) */
            xi[j] = xi[j] - gt * xi[k];
            for (r = 0; r < n_attr; ++r) {
                double *A = attr + (int64_t)r * attr_stride;
                A[k] = A[k] + (double)gt * A[j];
            }
        } else {
            /* eq. (6) */
            uint64_t half = xi[k] / 2;
            xi[j] = half;
            xi[k] = xi[k] - half;
            if (half == 0)
                counters[SDMO_CNT_ZEROED] += 1;
            for (r = 0; r < n_attr; ++r) {
                double *A = attr + (int64_t)r * attr_stride;
                double merged = A[k] + (double)gt * A[j];
                A[j] = merged;
                A[k] = merged;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* One timestep: the routine sequence of the workflow figure (Sec. 3.2).    */
/* ------------------------------------------------------------------------ */
int sdmo_step(uint64_t *xi, double *attr, int32_t n_attr, int64_t attr_stride,
              int64_t n_sd, const int32_t *cell_id, int32_t n_cell,
              const double *dv_per_cell, uint32_t *idx, int64_t *n_live,
              uint32_t *cell_start, const sdmo_params *p, uint64_t *counters,
              double *gamma_out, uint8_t *flag_out)
{
    int64_t n, q;
    double *u01 = (double *)malloc(sizeof(double) * (size_t)(n_sd + 1));
    double *prob = (double *)malloc(sizeof(double) * (size_t)(n_sd / 2 + 1));
    uint8_t *flag = (uint8_t *)malloc((size_t)(n_sd + 1));
    uint64_t local_counters[SDMO_CNT_N];
    int rc = 0;
    if (!counters) {
        memset(local_counters, 0, sizeof(local_counters));
        counters = local_counters;
    }

    /* step 0 */
    n = sdmo_remove_if_equal_0(idx, *n_live, xi);
    *n_live = n;
    /* step 1 */
    sdmo_urand(u01, n_sd, p->seed, p->run, p->step, SDMO_STREAM_SHUFFLE);
    if (sdmo_shuffle_per_cell(cell_start, idx, n, cell_id, n_cell, u01)) {
        rc = -1;
        goto done;
    }
    sdmo_flag_pairs(flag, cell_id, cell_start, idx, n);
    /* step 2 */
    sdmo_coalescence_kernel(prob, flag, attr, idx, n, p->kernel_id, p->kparams, p->table);
    sdmo_times_max(prob, xi, flag, idx, n);
    sdmo_normalize(prob, p->dt, dv_per_cell, cell_id, cell_start, flag, idx, n);
    /* step 3 */
    sdmo_urand(u01, n_sd / 2, p->seed, p->run, p->step, SDMO_STREAM_GAMMA);
    sdmo_compute_gamma(prob, u01, n / 2);
    sdmo_update_attributes(xi, attr, n_attr, attr_stride, prob, flag, idx, n,
                           counters);
    if (gamma_out) {
        for (q = 0; q < n_sd / 2; ++q)
            gamma_out[q] = q < n / 2 ? prob[q] : 0.0;
    }
    if (flag_out) {
        memcpy(flag_out, flag, (size_t)n);
        if (n_sd > n)
            memset(flag_out + n, 0, (size_t)(n_sd - n));
    }
done:
    free(u01);
    free(prob);
    free(flag);
    return rc;
}

/* Moments of the size spectrum per cell; the paper notes these are all a
 * CFD coupling needs (Sec. 5). */
int sdmo_moments(double *M, const uint64_t *xi, const double *volume,
                 const int32_t *cell_id, const uint32_t *idx, int64_t n_live,
                 int64_t n_sd, int32_t n_cell, const double *dv_per_cell)
{
    uint8_t *live = (uint8_t *)calloc((size_t)(n_sd + 1), 1);
    int64_t i, s;
    int32_t c;
    for (i = 0; i < n_live; ++i)
        live[idx[i]] = 1;
    for (c = 0; c < n_cell; ++c)
        M[3 * c] = M[3 * c + 1] = M[3 * c + 2] = 0.0;
    for (s = 0; s < n_sd; ++s) {
        double x, xv;
        if (!live[s])
            continue;
        c = cell_of(cell_id, (uint32_t)s);
        if (c < 0 || c >= n_cell) {
            free(live);
            return -1;
        }
        x = (double)xi[s];
        xv = x * volume[s];
        M[3 * c] = M[3 * c] + x;
        M[3 * c + 1] = M[3 * c + 1] + xv;
        M[3 * c + 2] = M[3 * c + 2] + xv * volume[s];
    }
    for (c = 0; c < n_cell; ++c) {
        M[3 * c] = M[3 * c] / dv_per_cell[c];
        M[3 * c + 1] = M[3 * c + 1] / dv_per_cell[c];
        M[3 * c + 2] = M[3 * c + 2] / dv_per_cell[c];
    }
    free(live);
    return 0;
}

void sdmo_reassign(int32_t *cell_id, int64_t n_sd, int32_t n_cell,
                   uint64_t seed, uint32_t step)
{
    int64_t s;
    for (s = 0; s < n_sd; ++s) {
        double u = sdmo_uniform(seed, 0, step, SDMO_STREAM_REASSIGN, (uint64_t)s);
        cell_id[s] = (int32_t)(u * (double)n_cell);
    }
}
