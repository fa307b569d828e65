/*
 * sdm_oracle.h -- reference (oracle) implementation of the Super-Droplet
 * Method coagulation step, written from Bartman & Arabas, "On the design of
 * Monte-Carlo particle coagulation solver interface: a CPU/GPU Super-Droplet
 * Method case study with PySDM" (arXiv:2101.06318).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is plain, single-threaded C99 in
 * IEEE binary64 with uint64 multiplicities.  It shares no code, header,
 * constant table or helper with the HIP library under paper_2101_06318_amd/;
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  The product path never calls it.
 *
 * Every routine mirrors one routine of the paper's backend API (Sec. 3.2,
 * Fig. "Algorithm workflow within a timestep") and works on host pointers.
 * Where the paper leaves a choice open, the reading taken is stated at the
 * routine; the same readings are listed in the repository design notes.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no fast-math), so
 * that every written floating-point operation is one correctly rounded
 * binary64 operation, in the written order.
 */
#ifndef SDM_ORACLE_H
#define SDM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Random streams (which Philox counter word 2 selects). */
enum { SDMO_STREAM_SHUFFLE = 0, SDMO_STREAM_GAMMA = 1, SDMO_STREAM_INIT = 2,
       SDMO_STREAM_REASSIGN = 3, SDMO_STREAM_MLP = 4, SDMO_STREAM_FY = 5,
       SDMO_STREAM_MERGE = 8 };

/* Coalescence kernels a(v1, v2). */
enum { SDMO_KERNEL_GOLOVIN = 0, SDMO_KERNEL_GEOMETRIC = 1,
       SDMO_KERNEL_CONSTANT = 2, SDMO_KERNEL_MULTIPLICATIVE = 3,
       SDMO_KERNEL_TABULATED = 4 };

/* Counter slots filled by sdmo_update_attributes (added to, never reset). */
enum { SDMO_CNT_PAIRS = 0,      /* flagged pairs visited                    */
       SDMO_CNT_COLLISIONS = 1, /* pairs with gamma-tilde > 0               */
       SDMO_CNT_CAPPED = 2,     /* gamma-tilde < gamma (multiple-coll. cap) */
       SDMO_CNT_ZEROED = 3,     /* equal-multiplicity split with xi_k == 1  */
       SDMO_CNT_GAMMA_GE2 = 4,  /* pairs with gamma >= 2                    */
       SDMO_CNT_N = 8 };

/* ---- Philox4x32-10 (Salmon et al., SC'11) -------------------------------
 * The paper names only CURandRTC as its uniform source; the reading taken
 * is the counter-based Philox4x32 with 10 rounds, counter
 * (e>>1, step, stream, run) and key (lo32(seed), hi32(seed)).  Element e
 * takes words 0-1 (even e) or 2-3 (odd e) of the output as a 64-bit word w,
 * high word first; the uniform is (w >> 11) * 2^-53 in [0, 1).          */
void     sdmo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                            uint32_t out[4]);
uint64_t sdmo_word(uint64_t seed, uint32_t run, uint32_t step,
                   uint32_t stream, uint64_t e);
double   sdmo_uniform(uint64_t seed, uint32_t run, uint32_t step,
                      uint32_t stream, uint64_t e);
/* urand (Step 1 and Step 3 of the workflow): u01[e] = U(seed,run,step,stream,e). */
void     sdmo_urand(double *u01, int64_t n, uint64_t seed, uint32_t run,
                    uint32_t step, uint32_t stream);

/* ---- Step 0: remove_if_equal_0 ------------------------------------------
 * Stable filter of the index list: keeps idx[i] with xi[idx[i]] > 0.
 * Returns the new live count.                                             */
int64_t  sdmo_remove_if_equal_0(uint32_t *idx, int64_t n_live,
                                const uint64_t *xi);

/* ---- Step 1: cell sort and shuffle_per_cell ------------------------------
 * sdmo_cell_sort: stable counting sort of idx[0:n_live] by cell_id[idx[i]];
 * cell_start[c] = number of live SDs in cells < c, for c in [0, n_cell].
 * sdmo_shuffle_per_cell: sort of idx[0:n_live] by the triple
 * (cell_id[s], floor(u01_by_sd[s] * 2^53), s) ascending -- the parallel
 * random-key sort the paper uses on the GPU, with the random key indexed by
 * the SD id s so that the result does not depend on the incoming order.
 * Both return 0, or -1 if a cell id lies outside [0, n_cell).            */
int      sdmo_cell_sort(uint32_t *cell_start, uint32_t *idx, int64_t n_live,
                        const int32_t *cell_id, int32_t n_cell);
/* The O(n) permutations of each cell (Sec. 3.2: the serial permutation
 * of the CPU backend, MergeShuffle for parallelism), applied to the live
 * SDs of each cell in their incoming order after a stable cell sort.
 * Random integer k uniform in [0, m): floor(U m) = (w m) >> 53 with w the
 * 53-bit word of U, exact in 128-bit integers.
 *  Fisher-Yates: for i = n-1 down to 1, k from draw (stream FY, element =
 *    the position cs + i), swap positions i and k of the cell.
 *  MergeShuffle: blocks of 16 positions from the cell's start get
 *    Fisher-Yates; then levels d = 1, 2, ...: blocks of 16 2^(d-1) are
 *    merged pairwise ([s, m) with [m, e), e = min(s + 16 2^d, cell end))
 *    by: i = s, j = m; repeat { coin = top bit of the draw (stream
 *    MERGE + 2d, element i); coin 0: stop if i == j; coin 1: stop if
 *    j == e, else swap i and j, j += 1; then i += 1 }; then for i < e:
 *    k uniform in [0, i - s] (stream MERGE + 2d + 1, element i), swap i and
 *    s + k.  Elements are global positions.  Returns -1 on a bad cell id. */
int      sdmo_shuffle_fisher_yates(uint32_t *cell_start, uint32_t *idx, int64_t n_live,
                                   const int32_t *cell_id, int32_t n_cell, uint64_t seed,
                                   uint32_t run, uint32_t step);
int      sdmo_shuffle_merge(uint32_t *cell_start, uint32_t *idx, int64_t n_live,
                            const int32_t *cell_id, int32_t n_cell, uint64_t seed,
                            uint32_t run, uint32_t step);
int      sdmo_shuffle_per_cell(uint32_t *cell_start, uint32_t *idx,
                               int64_t n_live, const int32_t *cell_id,
                               int32_t n_cell, const double *u01_by_sd);

/* flag_pairs: flag[i] = 1 iff position i opens a pair: i+1 < n_live, the SD
 * at i+1 lies in the same cell, and i - cell_start[cell] is even.         */
void     sdmo_flag_pairs(uint8_t *flag, const int32_t *cell_id,
                         const uint32_t *cell_start, const uint32_t *idx,
                         int64_t n_live);

/* ---- Step 2: collision probability, eq. (3) -----------------------------
 * Pair slot of the pair opened at flagged position i is floor(i/2); slots
 * [0, floor(n_live/2)) that no flagged position maps to hold 0.          */
/* Kernels: GOLOVIN kp[0](v1+v2); GEOMETRIC (the gravitational kernel);
 * CONSTANT kp[0]; MULTIPLICATIVE kp[0] v1 v2; TABULATED kp[0] times the
 * caller's table entry T[min(i1,i2)][max(i1,i2)] (table: n*n row-major),
 * i(v) = (bit pattern of v >> (52 - m)) - lo clamped to [0, n-1], with
 * lo = kp[1], n = kp[2], m = kp[3]; table is NULL for the other kernels. */
double   sdmo_kernel_value(int32_t kernel_id, const double *kparams,
                           const double *table, double v1, double v2);
void     sdmo_coalescence_kernel(double *pair_prob, const uint8_t *flag,
                                 const double *volume, const uint32_t *idx,
                                 int64_t n_live, int32_t kernel_id,
                                 const double *kparams, const double *table);
void     sdmo_times_max(double *pair_prob, const uint64_t *xi,
                        const uint8_t *flag, const uint32_t *idx,
                        int64_t n_live);
/* F(n) = ((n*n - n)/2) / floor(n/2) evaluated in integers (exact). */
uint64_t sdmo_pair_scale(uint64_t n);
void     sdmo_normalize(double *pair_prob, double dt, const double *dv_per_cell,
                        const int32_t *cell_id, const uint32_t *cell_start,
                        const uint8_t *flag, const uint32_t *idx,
                        int64_t n_live);

/* ---- Step 3: gamma and attribute update, eqs. (4)-(6) -------------------*/
void     sdmo_compute_gamma(double *pair_prob, const double *u01_by_slot,
                            int64_t n_slot);
void     sdmo_update_attributes(uint64_t *xi, double *attr, int32_t n_attr,
                                int64_t attr_stride, const double *gamma,
                                const uint8_t *flag, const uint32_t *idx,
                                int64_t n_live, uint64_t *counters);

/* ---- Whole timestep (the workflow figure, Steps 0-3) --------------------
 * Runs the routines above in the paper's order for one run.  u01 arrays are
 * generated by sdmo_urand from (seed, run, step).  Optional outputs (NULL to
 * skip): gamma_out[floor(N/2)] receives the slot gammas (0 for unused slots),
 * flag_out[N] the pair flags.  Returns 0, or -1 on a bad cell id.        */
typedef struct {
    double   dt;
    int32_t  kernel_id;
    double   kparams[4];
    uint64_t seed;
    uint32_t run;
    uint32_t step;
    const double *table;   /* TABULATED kernel only */
} sdmo_params;

int      sdmo_step(uint64_t *xi, double *attr, int32_t n_attr,
                   int64_t attr_stride, int64_t n_sd, const int32_t *cell_id,
                   int32_t n_cell, const double *dv_per_cell, uint32_t *idx,
                   int64_t *n_live, uint32_t *cell_start,
                   const sdmo_params *p, uint64_t *counters,
                   double *gamma_out, uint8_t *flag_out);

/* Per-cell moments M_k(c) = sum over live s in c of xi*v^k / dV_c, k=0,1,2,
 * summed in ascending SD-id order.  M is [n_cell][3].                    */
int      sdmo_moments(double *M, const uint64_t *xi, const double *volume,
                      const int32_t *cell_id, const uint32_t *idx,
                      int64_t n_live, int64_t n_sd, int32_t n_cell,
                      const double *dv_per_cell);

/* Project cube root (IEEE +,*,/ only) and the three-regime terminal
 * velocity used by the geometric (gravitational) kernel.                 */
double   sdmo_cbrt(double x);
double   sdmo_terminal_velocity(double r);

/* Cell reassignment used by the grid workload as a stand-in for advection:
 * cell_id[s] = floor(U(seed, 0, step, REASSIGN, s) * n_cell), n_cell a
 * power of two (exact).                                                   */
void     sdmo_reassign(int32_t *cell_id, int64_t n_sd, int32_t n_cell,
                       uint64_t seed, uint32_t step);

#ifdef __cplusplus
}
#endif
#endif
