// Host-side internals of the SDM library: context, sort plans, error
// reporting and launch helpers shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sdm.h"
#include "sdm_device.h"

namespace sdm {

// ------------------------------------------------------------ errors
void set_error(int code, const char *fmt, ...);
int fail(int code, const char *fmt, ...);  // sets the message, returns code

struct HipError {
    hipError_t e;
    const char *what;
};

#define SDM_HIP(call)                                                        \
    do {                                                                     \
        hipError_t _e = (call);                                              \
        if (_e != hipSuccess)                                                \
            throw ::sdm::HipError{_e, #call};                                \
    } while (0)

// Entry-point bodies: exceptions never cross the C boundary; every
// failure becomes a status code with a message.
#define SDM_TRY try {
#define SDM_CATCH                                                                     \
    }                                                                                 \
    catch (const ::sdm::HipError &he)                                                 \
    {                                                                                 \
        return ::sdm::fail(SDM_E_HIP, "%s: %s", he.what, hipGetErrorString(he.e));    \
    }                                                                                 \
    catch (const std::bad_alloc &)                                                    \
    {                                                                                 \
        return ::sdm::fail(SDM_E_NOMEM, "host allocation failed");                    \
    }                                                                                 \
    catch (...)                                                                       \
    {                                                                                 \
        return ::sdm::fail(SDM_E_STATE, "unexpected exception");                      \
    }                                                                                 \
    return SDM_OK;

#define REQUIRE(cond, ...)                                  \
    do {                                                    \
        if (!(cond))                                        \
            return ::sdm::fail(SDM_E_INVALID, __VA_ARGS__); \
    } while (0)

// ------------------------------------------------------------ engine plan
enum EngineMode { MODE_FUSED = 0, MODE_SHUFFLE = 1, MODE_CELLSORT = 2 };

// One SD's record between the tile and group kernels.  List modes: (shuffle
// key, id), 16 B.  Fused step: one 8-B word (layout RF_* below): the SD's
// slot within its tile, the bucket's low 5 bits, the 24 key bits below the
// bucket's, and upper-bound codes of its multiplicity and volume.  The
// group kernel draws the whole key again only for records whose stored
// bits tie, and reads xi and the attributes from the state only for pairs
// whose bound does not already rule a collision out.
struct __attribute__((aligned(16))) RecK {
    uint64_t key;
    uint32_t s;
    uint32_t pad;
};
constexpr int RF_BKT_SHIFT = 14;  // bits 0-13: slot within the tile (tiles <= 16384 slots)
constexpr int RF_KEY_SHIFT = 19;  // bits 14-18: bucket mod 32 (groups span <= 32 buckets)
constexpr int RF_XC_SHIFT = 43;   // bits 19-42: 24 key bits; bits 43-50: xi bound code
constexpr int RF_VC_SHIFT = 51;   // bits 51-63: volume bound code

// Pair that straddles two groups: the opener's record, written by the
// group holding it and completed by the finish kernel (which reads the two
// SDs' multiplicities and volumes from the state).
struct SeamRec {
    uint32_t s;
    uint32_t rank;
    int32_t cell;
    uint32_t cs;   // rank of the cell's first SD
    uint32_t n_c;  // live SDs in the cell
    uint32_t step; // the step the group kernel drew its numbers for
};

// Bucketed sort plan.  The live SDs of cell c are split by the top h[c]
// bits of their 53-bit shuffle key into 2^h[c] buckets.  The tile kernel
// sorts each tile of T SD slots by bucket in LDS and writes the tile's
// records contiguously, with its per-bucket offsets; the scan kernels turn
// the offsets into the global start rank of every bucket (hence of every
// group and cell); a group of consecutive buckets is then gathered from
// every tile and sorted by one workgroup.
struct Plan {
    int mode = 0;
    int64_t n_items = 0;  // SD slots (fused) or index capacity (list modes)
    int32_t n_cell = 0;
    int32_t B = 0, G = 0;
    int32_t tile = 0;     // SD slots per scatter tile (even, <= 1024 tile_ept)
    int32_t tile_ept = 0; // slots per tile-kernel thread (4, 8 or 16)
    int32_t n_tiles = 0;
    int32_t lhist = 0;    // tile-kernel histogram entries (B, or the largest local range)
    double bucket_target = 0, group_target = 0;  // effective plan targets
    // device tables
    int32_t *cell_h = nullptr;            // [C]
    int32_t *cell_bucket_base = nullptr;  // [C+1]
    int32_t *bucket_cell = nullptr;       // [B]
    uint8_t *sub_bits = nullptr;          // [B]
    int32_t *group_first = nullptr;       // [G+1]
    // per-cell run description (batched plans); null for single-run plans
    uint32_t *seg_off = nullptr;          // [C+1] SD slot offsets
    uint32_t *seg_len = nullptr;          // [C] SD slots of each run
    int32_t *seg_run = nullptr;           // [C]
    int32_t *seg_kernel = nullptr;        // [C] index into kernel table
    double *seg_dv = nullptr;             // [C]
    KernelDesc *kernels = nullptr;        // [n_kernels]
    // batched plans: tile t holds SDs of runs whose buckets are
    // [tile_lb[t], tile_lb[t] + tile_nb[t]); its exclusive offsets of those
    // buckets and its total (tile_nb[t] + 1 entries) sit at tile_loff[t] in
    // tile_off.  bk_ta[b] tiles lie wholly below bucket b, bk_tc[b] begin
    // below it.  Null for the other plans (dense tables).
    int32_t *tile_lb = nullptr;           // [n_tiles]
    int32_t *tile_nb = nullptr;           // [n_tiles]
    uint32_t *tile_loff = nullptr;        // [n_tiles]
    int32_t *bk_ta = nullptr;             // [B+1]
    int32_t *bk_tc = nullptr;             // [B+1]
    // workspace
    uint16_t *tile_off = nullptr;         // [n_tiles][B+1], or the batched plans' local tables
    uint16_t *tile_offT = nullptr;        // [B+1][n_tiles] (bucket-major copy; dense plans)
    // records in tile-local bucket order, [n_tiles * tile]
    RecK *rec_k = nullptr;                // list modes: (key, id)
    uint64_t *rec_f = nullptr;            // fused mode records (8 B)
    uint32_t chunk = 0;                   // records per LDS staging pass of the tile kernel
    int gept = 0;                         // records per group-kernel thread (4 or 8)
    bool whole_cells = false;             // every group holds whole cells
    uint32_t *n_acc = nullptr;            // [0] live total, [3] finish-kernel done counter
    uint32_t *bucket_start = nullptr;     // [B+1] global start rank per bucket
    uint32_t *cell_start_ws = nullptr;    // [C+1]
    int64_t *n_live_ws = nullptr;         // [1]
    uint64_t *sk = nullptr;               // [2 n_items + 8] global-sort scratch
    uint32_t *ss = nullptr;
    uint32_t *sb = nullptr;
    SeamRec *seam_open = nullptr;         // [G]
    SeamRec *seam_close = nullptr;        // [G]
    uint32_t *seam_state = nullptr;       // [G]
    uint32_t *group_tot = nullptr;        // [G]
    uint32_t *group_stats = nullptr;      // [G][5] collision statistics
    std::vector<void *> allocs;
};

struct PlanKey {
    int mode;
    int64_t n_items;
    int32_t n_cell;
    int64_t expected_milli;
    bool operator<(const PlanKey &o) const
    {
        return std::tie(mode, n_items, n_cell, expected_milli) <
               std::tie(o.mode, o.n_items, o.n_cell, o.expected_milli);
    }
};

}  // namespace sdm

struct sdm_batch {
    std::vector<sdm_segment> segs;
    int64_t n_items = 0;       // SD slots covered (last offset + n_sd, rounded up to even)
    int schedule = 0;
    sdm::Plan *plan = nullptr;
};

struct sdm_ctx {
    int device = 0;
    int64_t n_sd_max = 0;
    int32_t n_cell_max = 0;
    int32_t n_attr_max = 0;
    uint32_t *err_dev = nullptr;       // device error flags
    uint32_t *tmp_u32 = nullptr;       // [n_sd_max + 64] compaction scratch
    uint32_t *tile_cnt = nullptr;      // [tiles + 1]
    std::map<sdm::PlanKey, sdm::Plan *> plans;
    int32_t dbg_bucket_target = 0;     // testing: expected SDs per bucket
    int32_t dbg_group_cap = -1;        // testing: force the global-memory sort
    float *mlp_part = nullptr;         // [mlp_part_rows][n_params] backward partial sums
    int32_t mlp_part_rows = 0;
};

namespace sdm {

// Coalescence kernel descriptors (sdm_capi.hip): check_kernel validates an
// sdm_kernel on the host (returns SDM_OK or a failure with a message naming
// `what`); kernel_desc copies it for the device.
int check_kernel(const sdm_kernel &k, const char *what);
KernelDesc kernel_desc(const sdm_kernel &k);

// engine entry points (sdm_engine.hip)
Plan *get_plan(sdm_ctx *ctx, int mode, int64_t n_items, int32_t n_cell,
               double expected_per_cell);
void free_plan(Plan *p);

struct StepInputs {
    // items
    int64_t n_sd = 0;
    const int64_t *n_live_in = nullptr;  // list modes
    const uint32_t *idx_in = nullptr;    // list modes
    uint64_t *xi = nullptr;
    double *attr = nullptr;
    int32_t n_attr = 0;
    int64_t stride = 0;
    const int32_t *cell_id = nullptr;
    const double *u01 = nullptr;         // shuffle mode keys (may be null)
    // rng
    uint64_t seed = 0;
    uint32_t run = 0;
    uint32_t step = 0;
    const uint32_t *step_dev = nullptr;
    uint32_t *step_advance = nullptr;
    // physics (fused)
    double dt = 0;
    const double *dv_cell = nullptr;
    double dv = 0;
    KernelDesc kern{};
    // outputs
    uint32_t *idx_out = nullptr;
    uint32_t *cell_start = nullptr;
    int64_t *n_live_out = nullptr;
    uint64_t *counters = nullptr;
    double *gamma_out = nullptr;
    bool slot_cell_local = false;
    hipEvent_t events[4] = {nullptr, nullptr, nullptr, nullptr};
};

void engine_run(sdm_ctx *ctx, Plan *plan, const StepInputs &in, hipStream_t stream);

// batched ensembles (sdm_engine.hip)
int n_schedules();
// What a plan's launches depend on: schedules giving equal shapes are the same.
struct PlanShape {
    int32_t B, G, tile, n_tiles, tile_ept, gept;
    uint32_t chunk;
    double bucket_target, group_target;
    bool operator==(const PlanShape &o) const
    {
        return B == o.B && G == o.G && tile == o.tile && n_tiles == o.n_tiles &&
               tile_ept == o.tile_ept && gept == o.gept && chunk == o.chunk &&
               bucket_target == o.bucket_target && group_target == o.group_target;
    }
};
PlanShape shape_of(const Plan *p);
Plan *build_batch_plan(sdm_ctx *ctx, const std::vector<sdm_segment> &segs, int64_t n_items,
                       int schedule);

}  // namespace sdm
