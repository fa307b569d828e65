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

// ------------------------------------------------------------ engine plan
enum EngineMode { MODE_FUSED = 0, MODE_SHUFFLE = 1, MODE_CELLSORT = 2 };

// Records carried through the sort: one slot per SD.
struct SeamRec {
    uint64_t xi;
    double v;
    uint32_t s;
    uint32_t rank;
    int32_t cell;
    uint32_t pad;
};

// Bucketed sort plan.  The live SDs of cell c are split by the top h[c]
// bits of their 53-bit shuffle key into 2^h[c] buckets; each bucket owns a
// fixed region of cap slots in the record arrays (records beyond the
// capacity go to an overflow list).  Groups of consecutive buckets are
// sorted by one workgroup each.
struct Plan {
    int mode = 0;
    int64_t n_items = 0;  // SD slots (fused) or index capacity (list modes)
    int32_t n_cell = 0;
    int32_t B = 0, G = 0;
    int32_t lds_bins = 0;
    uint32_t S = 0;  // total record slots
    // device tables
    int32_t *cell_h = nullptr;            // [C]
    int32_t *cell_bucket_base = nullptr;  // [C+1]
    int32_t *bucket_cell = nullptr;       // [B]
    uint32_t *slot_base = nullptr;        // [B+1]
    uint8_t *sub_bits = nullptr;          // [B]
    int32_t *group_first = nullptr;       // [G+1]
    // per-cell run description (batched plans); null for single-run plans
    uint32_t *seg_off = nullptr;          // [C+1] SD slot offsets
    int32_t *seg_run = nullptr;           // [C]
    int32_t *seg_kernel = nullptr;        // [C] index into kernel table
    double *seg_dv = nullptr;             // [C]
    KernelDesc *kernels = nullptr;        // [n_kernels]
    // workspace
    uint32_t *cursor = nullptr;           // [B] (zero between launches)
    uint32_t *rank_off = nullptr;         // [B+1]
    uint32_t *cell_start_ws = nullptr;    // [C+1] (batched plans)
    int64_t *n_live_ws = nullptr;         // [1]
    uint32_t *ticket = nullptr;           // [1]
    uint64_t *rec_key = nullptr;          // [S]
    uint32_t *rec_s = nullptr;            // [S]
    uint64_t *rec_xi = nullptr;           // [S] (fused)
    double *rec_v = nullptr;              // [S] (fused)
    uint32_t *ov_count = nullptr;         // [1]
    uint64_t *ov_key = nullptr;           // [n_items]
    uint32_t *ov_s = nullptr;             // [n_items]
    uint32_t *ov_bucket = nullptr;        // [n_items]
    uint64_t *sk = nullptr;               // [2 n_items] slow-path scratch
    uint32_t *ss = nullptr;               // [2 n_items]
    uint32_t *sb = nullptr;               // [2 n_items]
    SeamRec *seam_open = nullptr;         // [G]
    SeamRec *seam_close = nullptr;        // [G]
    uint32_t *seam_state = nullptr;       // [G]
    uint32_t *group_tot = nullptr;        // [G]
    std::vector<void *> allocs;
    int group_threads = 512;
    int group_ept = 6;
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

struct sdm_ctx {
    int device = 0;
    int64_t n_sd_max = 0;
    int32_t n_cell_max = 0;
    int32_t n_attr_max = 0;
    uint32_t *err_dev = nullptr;       // device error flags
    uint32_t *tmp_u32 = nullptr;       // [n_sd_max + 64] compaction scratch
    uint32_t *tile_cnt = nullptr;      // [tiles + 1]
    std::map<sdm::PlanKey, sdm::Plan *> plans;
    int32_t dbg_bucket_cap = 0;        // testing: force tiny bucket regions
    int32_t dbg_group_cap = -1;        // testing: force the global-memory sort
};

namespace sdm {

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

}  // namespace sdm
