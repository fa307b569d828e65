/*
 * sdm.h -- C ABI of the MI355X (gfx950) Super-Droplet Method coagulation
 * library.  The routine set follows the backend API of Bartman & Arabas,
 * "On the design of Monte-Carlo particle coagulation solver interface: a
 * CPU/GPU Super-Droplet Method case study with PySDM" (arXiv:2101.06318),
 * Sec. 3: four data structures (Storage, IndexedStorage, Index,
 * PairIndicator) and the routines of the timestep workflow figure.
 *
 * Conventions (every entry point):
 *  - Return value: SDM_OK (0) or a negative sdm_status.  On an error nothing
 *    has been enqueued on the stream and sdm_last_error() (thread-local)
 *    describes it.
 *  - Pointers named *_dev or documented as "device" are device pointers into
 *    memory the caller owns (e.g. torch tensors' data_ptr()).  The library
 *    never frees or retains them after the call returns.  All device work is
 *    enqueued asynchronously on the caller's hipStream_t; no call blocks the
 *    host except sdm_create, sdm_destroy, sdm_prepare_step, sdm_batch_create,
 *    sdm_batch_destroy, sdm_autotune and sdm_read_errors.
 *  - Counts that change on the device (the live count n_live) stay on the
 *    device as int64_t*, so sequences of calls can be captured in a HIP graph
 *    (after a first eager call with the same shapes; see sdm_prepare_step).
 *  - Argument order: outputs, then in/out, then inputs, as the paper's
 *    intent comments in the workflow figure.
 *  - Types: sizes int64_t; SD ids uint32_t; cell ids int32_t;
 *    multiplicities xi uint64_t; attributes double, laid out row-major as
 *    attr[n_attr][attr_stride] (structure of arrays, Sec. 3.1); row 0 is the
 *    particle volume [m^3] the coalescence kernel reads.
 *  - Device-side anomalies are not call errors.  Collision statistics go
 *    into an optional caller-provided uint64_t counters_dev[8] (indices
 *    SDM_CNT_*, added to, never reset); malformed device data (a cell id out
 *    of range) is recorded in the context and reported by sdm_read_errors().
 *
 * Uniform random numbers (the paper names only its CURandRTC source): U =
 * (w >> 11) * 2^-53, w the 64-bit word of element e of Philox4x32-10 with
 * counter (e >> 1, step, stream, run) and key (lo32(seed), hi32(seed));
 * even e takes output words 0-1, odd e words 2-3 (high word first).
 */
#ifndef SDM_H
#define SDM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDM_ABI_VERSION 3

typedef enum {
    SDM_OK = 0,
    SDM_E_INVALID = -1,      /* null pointer, size or enum out of range      */
    SDM_E_HIP = -2,          /* HIP runtime or launch error                  */
    SDM_E_NOMEM = -3,        /* device allocation failed                     */
    SDM_E_UNSUPPORTED = -4,  /* size beyond what the context was created for */
    SDM_E_STATE = -5         /* context misuse                               */
} sdm_status;

/* Random streams: Philox counter word 2. */
enum { SDM_STREAM_SHUFFLE = 0, SDM_STREAM_GAMMA = 1, SDM_STREAM_INIT = 2,
       SDM_STREAM_REASSIGN = 3, SDM_STREAM_MLP = 4 };

/* Coalescence kernels a(v1, v2); p[] are the kernel parameters.
 *  GOLOVIN        b (v1 + v2)                      p[0] = b [1/s]
 *  GEOMETRIC      E pi (r1 + r2)^2 |w(r1) - w(r2)| p[0] = E (efficiency)
 *                 r = cbrt(0.75 v / pi) (Newton cube root, 8 IEEE steps),
 *                 w(r) = 1.19e8 r^2 (r < 8e3/1.19e8 m = 67.2 um),
 *                 8e3 r (r < (201/8e3)^2 m = 631 um), 201 sqrt(r)
 *                 otherwise [m/s]: each law up to where it meets the next
 *  CONSTANT       p[0]
 *  MULTIPLICATIVE p[0] v1 v2
 *  TABULATED      p[0] T[min(i1, i2)][max(i1, i2)]: any kernel, tabulated
 *                 by the caller on a binary-logarithmic grid of volumes.
 *                 i(v) = code(v) - lo clamped to [0, n - 1], where code(v)
 *                 is the IEEE-754 bit pattern of v read as an unsigned
 *                 integer and shifted right by 52 - m (2^m cells per
 *                 octave: cell code c holds the volumes whose pattern
 *                 starts with c); lo = p[1], n = p[2], m = p[3] (integers
 *                 held in doubles; 1 <= n <= 4096, 0 <= m <= 12).  T is
 *                 table[n * n], row-major, read only on or above the
 *                 diagonal, so the kernel is symmetric.  Only integer
 *                 operations pick the cell, so every backend gives the same
 *                 bits.  The fused step rules out no pair by a bound for
 *                 this kernel: every pair reads its SDs.
 * (Golovin, constant and multiplicative: Sec. 2.1; gravitational: Sec. 4;
 * the tabulated form is the plug-in point for the general kernels Sec. 5
 * names as an extension.) */
enum { SDM_KERNEL_GOLOVIN = 0, SDM_KERNEL_GEOMETRIC = 1,
       SDM_KERNEL_CONSTANT = 2, SDM_KERNEL_MULTIPLICATIVE = 3,
       SDM_KERNEL_TABULATED = 4 };

/* Counter slots (uint64_t counters_dev[8]). */
enum { SDM_CNT_PAIRS = 0,      /* flagged pairs visited                      */
       SDM_CNT_COLLISIONS = 1, /* pairs with gamma-tilde > 0                 */
       SDM_CNT_CAPPED = 2,     /* gamma-tilde < gamma (eq. 4 cap active)     */
       SDM_CNT_ZEROED = 3,     /* eq. (6) split with xi_k = 1: xi_j -> 0     */
       SDM_CNT_GAMMA_GE2 = 4,  /* pairs with gamma >= 2                      */
       SDM_CNT_FALLBACK = 5,   /* cells outside the surrogate's input hull   */
       SDM_CNT_N = 8 };

typedef struct sdm_ctx sdm_ctx;
typedef struct sdm_batch sdm_batch;

typedef struct {
    int32_t id;              /* SDM_KERNEL_*                                 */
    int32_t reserved;
    double  p[4];            /* kernel parameters (see above)                */
    const double *table;     /* SDM_KERNEL_TABULATED: device double[n * n],  */
                             /* caller-owned, read while the calls (or a     */
                             /* graph that captured them) run; else NULL     */
} sdm_kernel;

typedef struct {
    uint64_t        seed;
    uint32_t        run;
    uint32_t        step;    /* timestep index; ignored if step_dev != NULL  */
    const uint32_t *step_dev;/* optional device pointer to the step index,   */
                             /* so a captured graph can advance it           */
} sdm_rng;

/* ---------------------------------------------------------------- setup */
int         sdm_abi_version(void);
const char *sdm_last_error(void);

/* Creates a context on the current HIP device for up to n_sd_max SD slots,
 * n_cell_max cells and n_attr_max attribute rows.  The context owns its
 * device workspace (sort buckets, scan buffers, counters).  Blocking. */
int sdm_create(sdm_ctx **ctx, int64_t n_sd_max, int32_t n_cell_max,
               int32_t n_attr_max);
int sdm_destroy(sdm_ctx *ctx);

/* Reads and clears the context's device error flags (blocking).
 * *flags bit 0: a cell id outside [0, n_cell) was seen (that SD was left out
 * of the sort). */
int sdm_read_errors(sdm_ctx *ctx, uint32_t *flags);

/* Testing hook: rebuilds the sort plans with bucket_target expected SDs
 * per key bucket (0 = automatic, 2048) and a group capacity of group_cap
 * records (< 0 = automatic), so that cells spanning many groups, seams and
 * the global-memory sort path run on ordinary inputs.  Results are
 * identical; only speed changes.  Blocking. */
int sdm_set_plan_limits(sdm_ctx *ctx, int32_t bucket_target, int32_t group_cap);

/* ------------------------------------------------------------ R2 urand */
/* u01[e] = U(seed, run, step, stream_id, e) for e in [0, n).
 * u01: device, n doubles, written. */
int sdm_urand(sdm_ctx *ctx, double *u01, int64_t n, const sdm_rng *rng,
              uint32_t stream_id, hipStream_t stream);

/* --------------------------------------------------- Step 0 (R1) */
/* Stable removal of zero-multiplicity SDs from the Index (Sec. 3.2, Step 0).
 * idx: device uint32[n_sd_max], in/out (entries [0, *n_live_dev) used);
 * n_live_dev: device int64, in/out; xi: device uint64 indexed by SD id. */
int sdm_remove_if_equal_0(sdm_ctx *ctx, uint32_t *idx, int64_t *n_live_dev,
                          const uint64_t *xi, hipStream_t stream);

/* Largest Index sdm_remove_if_equal_0_noalloc accepts (4,194,304 ids). */
#define SDM_NOALLOC_MAX_IDS ((int64_t)1 << 22)

/* Step 0 for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops or harnesses that forbid hipMalloc): the
 * same result as sdm_remove_if_equal_0, with no context and no allocation
 * of any kind.  Its scratch is one fixed library-owned device array of
 * SDM_NOALLOC_MAX_IDS + 64 ids and 2112 tile counts (16 MiB + 8.3 KiB),
 * which every GPU the library runs on holds until the process ends; its
 * address is resolved once per device on the first call (with that device
 * current).  All calls on one GPU share that array and it keeps the last
 * call's contents (nothing in it needs to start at zero), so calls that
 * overlap on one GPU (two streams, two host threads) race: serialise them.
 * idx: device uint32[n_sd_max], in/out; n_live_dev: device int64, in/out,
 * at most n_sd_max (a larger value is read as n_sd_max); xi: device uint64
 * by SD id.  The current device must be the device of idx and stream.
 * Errors: SDM_E_INVALID for a null pointer or n_sd_max outside
 * [1, SDM_NOALLOC_MAX_IDS]; SDM_E_HIP if the scratch address cannot be
 * resolved or a launch fails. */
int sdm_remove_if_equal_0_noalloc(uint32_t *idx, int64_t *n_live_dev, const uint64_t *xi,
                                  int64_t n_sd_max, hipStream_t stream);

/* --------------------------------------------------- Step 1 (R3, R4) */
/* Stable counting sort of idx[0:n_live] by cell_id[idx[i]] (the Index's
 * sort-by-key on the cell id, Sec. 3.1).
 * cell_start: device uint32[n_cell+1], out: cell_start[c] = number of live
 * SDs in cells < c.  idx: in/out.  cell_id: device int32 by SD id. */
int sdm_cell_sort(sdm_ctx *ctx, uint32_t *cell_start, uint32_t *idx,
                  const int64_t *n_live_dev, const int32_t *cell_id,
                  int32_t n_cell, hipStream_t stream);

/* shuffle_per_cell (Sec. 3.2, Step 1): sorts idx[0:n_live] by
 * (cell_id[s], floor(u_s * 2^53), s) ascending, the random-key sort the
 * paper uses on the GPU.  u_s = u01_by_sd[s] (device double by SD id) or,
 * if u01_by_sd is NULL, U(rng, SDM_STREAM_SHUFFLE, s) generated inline
 * (values outside [0, 1) are clamped to that range).  idx entries must be
 * valid SD ids (< n_sd_max).
 * cell_start: out as above.  cell_idx: optional device int32[n_cell] cell
 * traversal order (scheduling hint only; results do not depend on it). */
int sdm_shuffle_per_cell(sdm_ctx *ctx, uint32_t *cell_start, uint32_t *idx,
                         const int64_t *n_live_dev, const int32_t *cell_idx,
                         const int32_t *cell_id, int32_t n_cell,
                         const double *u01_by_sd, const sdm_rng *rng,
                         hipStream_t stream);

/* The O(n) permutations of each cell that Sec. 3.2 names besides sorting
 * by random keys: the serial permutation of the CPU backend (Fisher-Yates,
 * after Appendix A of the original SDM paper) and MergeShuffle (Bacher et
 * al. 2015), which parallelises within a cell.  idx[0:n_live] is first
 * cell-sorted stably (as sdm_cell_sort), then each cell's segment, in that
 * order, is permuted in place.  A random integer uniform in [0, m) is
 * floor(U m) = (w m) >> 53, w the 53-bit word of U(rng, stream, element).
 *  SDM_SHUFFLE_FISHER_YATES: for i = n-1 down to 1 (n the cell's size),
 *    k uniform in [0, i] (stream 5, element = global position cs + i),
 *    swap the cell's positions i and k.
 *  SDM_SHUFFLE_MERGE: Fisher-Yates (as above) on blocks of 16 positions
 *    from the cell's start; then for d = 1, 2, ... the blocks of 16 2^(d-1)
 *    are merged pairwise, [s, m) with [m, e), e = min(s + 16 2^d, cell
 *    end): i = s, j = m; repeat { coin = top bit of the word of (stream
 *    8 + 2d, element i); coin 0: stop if i == j; coin 1: stop if j == e,
 *    else swap i and j, j += 1; i += 1 }; then for each remaining i < e: k
 *    uniform in [0, i - s] (stream 9 + 2d, element i), swap i and s + k.
 *    Elements are global positions.
 * Both give uniformly random permutations (pinned by exact enumeration and
 * frequency tests) but not the permutation of sdm_shuffle_per_cell.  Fisher-
 * Yates runs one thread per cell; MergeShuffle one launch per level.  Same
 * arguments as sdm_cell_sort plus the method and the random numbers. */
enum { SDM_SHUFFLE_FISHER_YATES = 1, SDM_SHUFFLE_MERGE = 2 };
int sdm_shuffle_variant(sdm_ctx *ctx, int32_t method, uint32_t *cell_start, uint32_t *idx,
                        const int64_t *n_live_dev, const int32_t *cell_id, int32_t n_cell,
                        const sdm_rng *rng, hipStream_t stream);

/* flag_pairs (PairIndicator, Sec. 3.1; GPU listing Fig. 3):
 * pair_flag[i] = i+1 < n_live && cell(idx[i+1]) == cell(idx[i]) &&
 *                (i - cell_start[cell(idx[i])]) even.
 * pair_flag: device uint8[n_sd_max], out (entries [0, n_live)). */
int sdm_flag_pairs(sdm_ctx *ctx, uint8_t *pair_flag, const int32_t *cell_id,
                   const int32_t *cell_idx, const uint32_t *cell_start,
                   const uint32_t *idx, const int64_t *n_live_dev,
                   hipStream_t stream);

/* --------------------------------------------------- Step 2 (R5-R7), eq. 3 */
/* The pair opened at flagged position i owns slot floor(i/2) of pair_prob
 * (device double[n_sd_max/2]); slots [0, floor(n_live/2)) with no flagged
 * position are set to 0 by coalescence_kernel and left alone by the rest.
 * coalescence_kernel: p = a(v_j, v_k).
 * times_max:          p = p * max(xi_j, xi_k).
 * normalize:          p = p * ((dt / dv_per_cell[c]) * F(n_c)),
 *                     F(n) = ((n^2 - n)/2) / floor(n/2) in integers.
 * pair_rate:          the three in one pass, same result bit for bit.      */
int sdm_coalescence_kernel(sdm_ctx *ctx, double *pair_prob,
                           const uint8_t *pair_flag, const double *volume,
                           const uint32_t *idx, const int64_t *n_live_dev,
                           const sdm_kernel *kernel, hipStream_t stream);
int sdm_times_max(sdm_ctx *ctx, double *pair_prob, const uint64_t *xi,
                  const uint8_t *pair_flag, const uint32_t *idx,
                  const int64_t *n_live_dev, hipStream_t stream);
int sdm_normalize(sdm_ctx *ctx, double *pair_prob, double dt,
                  const double *dv_per_cell, const int32_t *cell_id,
                  const int32_t *cell_idx, const uint32_t *cell_start,
                  const uint8_t *pair_flag, const uint32_t *idx,
                  const int64_t *n_live_dev, hipStream_t stream);
int sdm_pair_rate(sdm_ctx *ctx, double *pair_prob, double dt,
                  const double *dv_per_cell, const uint8_t *pair_flag,
                  const double *volume, const uint64_t *xi,
                  const int32_t *cell_id, const uint32_t *cell_start,
                  const uint32_t *idx, const int64_t *n_live_dev,
                  const sdm_kernel *kernel, hipStream_t stream);

/* --------------------------------------------------- Step 3 (R8, R9) */
/* compute_gamma: pair_prob[q] = ceil(pair_prob[q] - phi_q) in place for
 * q in [0, floor(n_live/2)); phi_q = u01_by_slot[q] or, if NULL,
 * U(rng, SDM_STREAM_GAMMA, q). */
int sdm_compute_gamma(sdm_ctx *ctx, double *pair_prob,
                      const double *u01_by_slot, const sdm_rng *rng,
                      const int64_t *n_live_dev, hipStream_t stream);

/* update_attributes, eqs. (4)-(6): for every flagged i, j and k are the SDs
 * at i and i+1, swapped so that xi_j >= xi_k (a tie keeps j at i);
 * g = min(gamma, floor(xi_j/xi_k)) with gamma read from slot floor(i/2)
 * (NaN and values < 1 read as 0, >= 2^64 saturate); case 1 (xi_j - g xi_k >
 * 0): xi_j -= g xi_k, A_k += g A_j; case 2: xi_j = floor(xi_k/2),
 * xi_k -= xi_j, A_j = A_k = A_k + g A_j.  xi, attr: in/out, by SD id.
 * counters_dev: optional uint64[8]. */
int sdm_update_attributes(sdm_ctx *ctx, uint64_t *xi, double *attr,
                          int32_t n_attr, int64_t attr_stride,
                          const double *gamma, const uint8_t *pair_flag,
                          const uint32_t *idx, const int64_t *n_live_dev,
                          uint64_t *counters_dev, hipStream_t stream);

/* --------------------------------------------------- fused timestep */
/* State of one run (Sec. 3.1 state listing).  All pointers are device
 * pointers owned by the caller. */
typedef struct {
    int64_t   n_sd;          /* SD slots                                    */
    int32_t   n_cell;
    int32_t   n_attr;
    int64_t   attr_stride;   /* >= n_sd                                     */
    uint64_t *xi;            /* [n_sd]            in/out                    */
    double   *attr;          /* [n_attr][stride]  in/out                    */
    const int32_t *cell_id;  /* [n_sd] or NULL (every SD in cell 0)         */
    uint32_t *idx;           /* [n_sd]            out: sorted live SDs      */
    int64_t  *n_live_dev;    /* [1]               out                       */
    uint32_t *cell_start;    /* [n_cell+1]        out                       */
    uint64_t *counters_dev;  /* [8] or NULL       added to                  */
    double   *gamma_out;     /* [n_sd/2] or NULL: slot gammas (diagnostic)  */
} sdm_state;

typedef struct {
    double            dt;            /* [s]                                 */
    const double     *dv_per_cell;   /* device [n_cell], or NULL => dv      */
    double            dv;            /* [m^3] used when dv_per_cell is NULL */
    sdm_kernel        kernel;
    sdm_rng           rng;
    uint32_t         *step_advance;  /* optional device counter incremented */
                                     /* by one at the end of the step       */
    double            expected_per_cell; /* planning hint (0 => n_sd/n_cell)*/
    hipEvent_t        events[4];     /* optional (NULL entries skipped):    */
                                     /* recorded on the stream before the   */
                                     /* partition kernels (tile, column     */
                                     /* sums),                              */
                                     /* the group kernel, the finish kernel */
                                     /* and after it, for timing            */
} sdm_step_params;

/* One whole timestep (workflow figure, Steps 0-3) in four kernels (three
 * when every group of the plan holds one cell or whole cells and the plan
 * has at most 512 tiles: no column-sum kernel), with the
 * result of running the routines above in the paper's order with inline
 * random numbers: the live set is {s : xi[s] > 0} (Step 0), idx receives
 * the live SDs sorted by (cell, shuffle key, s), the pairs and slots are
 * those of flag_pairs, gamma draws U(rng, SDM_STREAM_GAMMA, slot).  The
 * incoming idx order is not read.  The first call for a given shape builds
 * the plan (allocating, not capturable); sdm_prepare_step does that
 * explicitly so the step can then be captured. */
int sdm_prepare_step(sdm_ctx *ctx, const sdm_state *st,
                     const sdm_step_params *p);
int sdm_step(sdm_ctx *ctx, const sdm_state *st, const sdm_step_params *p,
             hipStream_t stream);

/* --------------------------------------------------- batched ensemble */
/* One independent run of a batch: SD slots [offset, offset + n_sd) of the
 * batch state form one well-mixed cell (its own volume dv and kernel); the
 * run's random streams use Philox run word `run` and run-local SD ids and
 * pair slots, so every member gives exactly the result it gives alone. */
typedef struct {
    int64_t    offset;       /* first SD slot (even)                        */
    int64_t    n_sd;         /* SD slots of the run                         */
    double     dv;           /* [m^3]                                       */
    sdm_kernel kernel;
    uint32_t   run;          /* Philox run word                             */
    uint32_t   reserved;
} sdm_segment;

/* Creates a batch of n_seg runs (blocking; the batch owns its plan and
 * schedule tables until sdm_batch_destroy).  Segments must be sorted by
 * offset, non-overlapping, with even offsets; n_seg <= n_cell_max. */
int sdm_batch_create(sdm_ctx *ctx, sdm_batch **b, const sdm_segment *segs,
                     int32_t n_seg);
int sdm_batch_destroy(sdm_ctx *ctx, sdm_batch *b);

/* One timestep of every run of the batch in one four-kernel launch
 * sequence (graph-capturable after the first call).  st->n_cell must equal
 * the number of segments and st->cell_id is ignored; cell_start[r] receives
 * the first rank of run r, idx the sorted live SDs of every run (global SD
 * ids, run after run), gamma_out (optional) slot q of run r at
 * offset_r/2 + q.  p->dt and p->rng.seed/step/step_dev apply to all runs;
 * p->kernel, p->dv and p->rng.run are taken from the segments. */
int sdm_batch_step(sdm_ctx *ctx, sdm_batch *b, const sdm_state *st,
                   const sdm_step_params *p, hipStream_t stream);

/* Sets the batch's schedule to candidate `schedule` (0 <= schedule <
 * *n_schedules), or only reports the number of candidates when schedule < 0.
 * Blocking. */
int sdm_batch_set_schedule(sdm_ctx *ctx, sdm_batch *b, int32_t schedule,
                           int32_t *n_schedules);

/* Chooses the batch's block and segment schedule (key-bucket size, group
 * packing, tile-kernel slots per thread) by timing each distinct candidate
 * plan on the scratch state (which is advanced): two passes over the
 * candidates, the second in reverse order, each a warm-up step and `steps`
 * timed steps, the faster pass counting; or loads the choice from
 * cache_path (a text file keyed by the segment-size layout; NULL = no
 * cache) and stores it there.  Results never depend on the schedule.
 * Blocking; holds every candidate plan's workspace until it returns.
 * *chosen (may be NULL) receives the index of the chosen candidate. */
int sdm_autotune(sdm_ctx *ctx, sdm_batch *b, const sdm_state *scratch,
                 const sdm_step_params *p, int32_t steps, const char *cache_path,
                 int32_t *chosen);

/* --------------------------------------------------- moments */
/* M[c][k] = sum over live s in cell c of xi_s v_s^k / dV_c, k = 0, 1, 2.
 * Needs idx sorted by cell with cell_start (as after a step).  M: device
 * double[n_cell][3], out.  Sum order is fixed (deterministic). */
int sdm_moments(sdm_ctx *ctx, double *M, const uint64_t *xi,
                const double *volume, const uint32_t *idx,
                const uint32_t *cell_start, int32_t n_cell,
                const double *dv_per_cell, double dv, hipStream_t stream);

/* Grid workload driver (advection stand-in): cell_id[s] =
 * floor(U(seed, 0, step, SDM_STREAM_REASSIGN, s) * n_cell), n_cell a power
 * of two.  cell_id: device int32[n_sd], out. */
int sdm_reassign(sdm_ctx *ctx, int32_t *cell_id, int64_t n_sd, int32_t n_cell,
                 const sdm_rng *rng, hipStream_t stream);

/* --------------------------------------------------- moment surrogate */
/* A learned model of one cell's coagulation over dt in terms of its bulk
 * moments only (the paper's outlook, Sec. 5: a coupled fluid solver needs
 * statistical moments of the spectrum, not the particles).
 *
 * Network: x[5] -> 128 -> 128 -> 128 -> y[3]; layer l computes
 * z = W_l a + b_l, GELU(z) = z Phi(z) (exact erf form) after each hidden
 * layer, linear output.  x = standardised (log M0, log M1, log M2, dt,
 * kernel id) of a cell; y = standardised relative moment tendencies
 * (M_k(t + dt) - M_k(t)) / (M_k(t) dt).  Arithmetic: every matmul takes
 * bfloat16 operands (weights, x, activations, back-propagated errors,
 * rounded to nearest even) on the matrix cores with float32 accumulation;
 * bias adds, GELU, its derivative, loss, gradients and Adam are float32.
 *
 * Parameters: one flat float32 vector of SDM_MLP_N_PARAMS entries in the
 * order W1, b1, W2, b2, W3, b3, W4, b4, each W row-major [out][in]. */
#define SDM_MLP_N_PARAMS 34179
#define SDM_MLP_PACKED_BYTES 151552   /* bf16 weights in the kernels' order */
#define SDM_MLP_CACHE_FLOATS_PER_ROW 576

typedef struct {
    float *params;           /* device float[SDM_MLP_N_PARAMS]: fp32 masters */
    void  *packed;           /* device, SDM_MLP_PACKED_BYTES, 16-B aligned:  */
                             /* bf16 copy written by sdm_mlp_pack/_adam      */
} sdm_mlp;

typedef struct {
    float *m;                /* device float[SDM_MLP_N_PARAMS], start at 0   */
    float *v;                /* device float[SDM_MLP_N_PARAMS], start at 0   */
} sdm_mlp_opt;

typedef struct {
    double  lr, beta1, beta2, eps;  /* 1 - beta is formed in double, then */
                                    /* rounded to float for the kernel    */
    int32_t t;               /* 1-based step number (bias correction)        */
    int32_t reserved;
} sdm_adam_hp;

/* Rounds the fp32 masters to bf16 into w->packed.  Call after writing
 * w->params (sdm_mlp_adam repacks by itself). */
int sdm_mlp_pack(sdm_ctx *ctx, const sdm_mlp *w, hipStream_t stream);

/* y[B][3] = network(x[B][5]) (device float, row-major).  cache: NULL for
 * inference, or device float[ceil(B/16)*16 * SDM_MLP_CACHE_FLOATS_PER_ROW]
 * receiving, for sdm_mlp_backward, the derivative GELU'(z) of every hidden
 * unit and the bf16 activations the forward pass used (layout private
 * to the library).  B = 0 is a no-op. */
int sdm_mlp_forward(sdm_ctx *ctx, float *y, float *cache, const float *x, int64_t B,
                    const sdm_mlp *w, hipStream_t stream);

/* grad[SDM_MLP_N_PARAMS] (device float, overwritten) = d(sum_b,j dy[b][j]
 * y[b][j]) / d params, for the batch of the forward call that filled
 * cache from x.  Sums over the batch in a fixed order (deterministic).  The
 * first call with a batch needing more partial-sum rows than any before
 * allocates (blocking; not capturable). */
int sdm_mlp_backward(sdm_ctx *ctx, float *grad, const float *dy, const float *x,
                     const float *cache, int64_t B, const sdm_mlp *w, hipStream_t stream);

/* Mean-squared error over the B*3 outputs: dy = 2 (y - t) / (3B) and
 * *loss = sum (y - t)^2 / (3B) (device floats; loss may be NULL). */
int sdm_mlp_mse(sdm_ctx *ctx, float *dy, float *loss, const float *y, const float *t,
                int64_t B, hipStream_t stream);

/* One Adam step (Kingma & Ba) on w->params from grad, updating opt->m,
 * opt->v and, in the same kernel, each updated weight's bf16 copies in
 * w->packed (w->packed must hold a pack of the network, whose padding the
 * pack wrote: sdm_mlp_pack once after writing w->params). */
int sdm_mlp_adam(sdm_ctx *ctx, const sdm_mlp *w, const sdm_mlp_opt *opt, const float *grad,
                 const sdm_adam_hp *hp, hipStream_t stream);

/* Out-of-distribution test: fallback[b] = 1 when any feature x[b][i] lies
 * outside [lo[i], hi[i]] or is NaN (the per-feature box of the training
 * inputs), else 0.  lo, hi: host float[5] (copied).  counters_dev
 * (optional) gets the number of fallback rows added at SDM_CNT_FALLBACK. */
int sdm_hull_check(sdm_ctx *ctx, uint8_t *fallback, uint64_t *counters_dev, const float *x,
                   int64_t B, const float *lo, const float *hi, hipStream_t stream);

/* Joint out-of-distribution test of the surrogate's inputs (a cell it
 * cannot vouch for falls back to the particle method; Sec. 5 motivates a
 * moments-only coupling): fallback[b] = 1 when any feature x[b][i] lies
 * outside [lo[i], hi[i]] or is NaN, or, with an occupancy grid, when the
 * cell of (x[b][0], x[b][1], x[b][2]) holds no training input: cell index
 * k_i = floor((x[b][i] - glo[i]) * ginv[i]) clamped to [0, G - 1] (single
 * precision, in this order), occ[(k_0 G + k_1) G + k_2] != 0 for cells the
 * training inputs reached.  lo, hi: host float[5]; glo, ginv: host float[3]
 * (copied); occ: device uint8[G^3] or NULL (box only), 1 <= G <= 256.
 * counters_dev (optional) gets the number of fallback rows. */
int sdm_ood_check(sdm_ctx *ctx, uint8_t *fallback, uint64_t *counters_dev, const float *x,
                  int64_t B, const float *lo, const float *hi, const uint8_t *occ, int32_t G,
                  const float *glo, const float *ginv, hipStream_t stream);

/* The surrogate's fallback: particles rebuilt from a cell's moments, to be
 * advanced by the particle method (sdm_batch_step with one segment of
 * n_per_cell slots per cell) and measured again (sdm_moments).  For cell c
 * with select[c] != 0 (select NULL: every cell) and M0, M1, M2 > 0, slots
 * [c n, c n + n) (n = n_per_cell) receive n SDs at the standard-normal
 * quantiles z_i = sqrt(2) erfinv(2 (i + 1/2)/n - 1): volumes e^(sigma z_i)
 * scaled to the mean volume M1/M0, sigma chosen so that the SDs' own
 * M2 M0 / M1^2 equals the cell's (60 bisection steps; the set holds at
 * most n times the squared mean, so larger ratios are capped), every
 * multiplicity rint(M0 dv / n), at least 1: the cell's M0 up to that
 * rounding, M1 and M2 exactly.  Other cells' slots get multiplicity 0 and
 * volume 0.  M: device double[n_cell][3] (per unit volume, sdm_moments
 * layout); xi: device uint64[n_cell n]; v: device double[n_cell n]
 * (attribute row 0). */
int sdm_seed_from_moments(sdm_ctx *ctx, uint64_t *xi, double *v, const double *M,
                          const uint8_t *select, int32_t n_cell, int32_t n_per_cell, double dv,
                          hipStream_t stream);

/* M[c] = M_src[c] (all three moments) for cells with select[c] != 0.
 * M, M_src: device double[n][3]; select: device uint8[n]. */
int sdm_moments_merge(sdm_ctx *ctx, double *M, const double *M_src, const uint8_t *select,
                      int64_t n, hipStream_t stream);

/* Surrogate input of n cells: x[c] = ((log M0, log M1, log M2, dt,
 * kernel_id) - mean) / std with M: device double[n][3] (sdm_moments
 * layout), x: device float[n][5]; mean, std: host float[5] (copied). */
int sdm_mlp_features(sdm_ctx *ctx, float *x, const double *M, int64_t n, double dt,
                     int32_t kernel_id, const float *mean, const float *std,
                     hipStream_t stream);

/* Surrogate update of n cells: M[c][k] *= 1 + dt (y[c][k] std[k] + mean[k])
 * for cells with fallback[c] == 0 (fallback may be NULL); others are left
 * for the particle step.  M: device double[n][3]; y: device float[n][3];
 * mean, std: host float[3] (target standardisation, copied). */
int sdm_mlp_apply(sdm_ctx *ctx, double *M, const float *y, const uint8_t *fallback, int64_t n,
                  double dt, const float *mean, const float *std, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SDM_H */
