// Context management, error reporting and the fused timestep entry points
// of the C ABI (include/sdm.h).
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>

#include "sdm_internal.h"

namespace sdm {

static thread_local char g_err[512] = "";

void set_error(int code, const char *fmt, ...)
{
    (void)code;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace sdm

using namespace sdm;

// Zero fill by a kernel (not a memset node) so the call stays graph-safe.
__global__ void k_fill_zero_f64(double *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0.0;
}

static void destroy_ctx(sdm_ctx *c)
{
    if (!c)
        return;
    for (auto &kv : c->plans)
        free_plan(kv.second);
    c->plans.clear();
    if (c->err_dev)
        (void)hipFree(c->err_dev);
    if (c->tmp_u32)
        (void)hipFree(c->tmp_u32);
    if (c->tile_cnt)
        (void)hipFree(c->tile_cnt);
    if (c->mlp_part)
        (void)hipFree(c->mlp_part);
    delete c;
}

static int check_state(const sdm_ctx *ctx, const sdm_state *st, const sdm_step_params *p)
{
    REQUIRE(ctx && st && p, "null argument");
    REQUIRE(st->n_sd >= 0 && st->n_sd <= ctx->n_sd_max, "n_sd %lld out of range",
            (long long)st->n_sd);
    REQUIRE(st->n_cell >= 1 && st->n_cell <= ctx->n_cell_max, "n_cell %d out of range",
            st->n_cell);
    REQUIRE(st->n_attr >= 1 && st->n_attr <= ctx->n_attr_max, "n_attr %d out of range",
            st->n_attr);
    REQUIRE(st->attr_stride >= st->n_sd, "attr_stride < n_sd");
    REQUIRE(st->n_live_dev && st->cell_start, "state pointer is NULL");
    if (st->n_sd > 0) {  // an empty state may carry null arrays
        REQUIRE(st->xi && st->attr && st->idx, "state pointer is NULL");
        REQUIRE(st->n_cell == 1 || st->cell_id, "cell_id is NULL with n_cell > 1");
        REQUIRE(((uintptr_t)st->xi & 15) == 0, "xi must be 16-byte aligned");
    }
    REQUIRE(p->dv_per_cell || p->dv > 0, "need dv_per_cell or dv > 0");
    if (int rc = check_kernel(p->kernel, "kernel"))
        return rc;
    REQUIRE(std::isfinite(p->dt) && p->dt >= 0, "dt invalid");
    return SDM_OK;
}

namespace sdm {

int check_kernel(const sdm_kernel &k, const char *what)
{
    if (k.id < SDM_KERNEL_GOLOVIN || k.id > SDM_KERNEL_TABULATED)
        return fail(SDM_E_INVALID, "%s: unknown kernel id %d", what, k.id);
    if (k.id == SDM_KERNEL_TABULATED) {
        const double n = k.p[2], m = k.p[3], lo = k.p[1];
        if (!k.table)
            return fail(SDM_E_INVALID, "%s: tabulated kernel without a table", what);
        if (!(n >= 1 && n <= 4096 && n == std::floor(n)))
            return fail(SDM_E_INVALID, "%s: table size p[2] must be an integer in [1, 4096]",
                        what);
        if (!(m >= 0 && m <= 12 && m == std::floor(m)))
            return fail(SDM_E_INVALID, "%s: cells per octave p[3] must be 2^m, m in [0, 12]",
                        what);
        if (!(lo >= 0 && lo < 4096.0 * 4096.0 && lo == std::floor(lo)))
            return fail(SDM_E_INVALID, "%s: first cell code p[1] invalid", what);
    }
    return SDM_OK;
}

KernelDesc kernel_desc(const sdm_kernel &k)
{
    KernelDesc d{};
    d.id = k.id;
    d.reserved = 0;
    for (int i = 0; i < 4; ++i)
        d.p[i] = k.p[i];
    d.table = k.id == SDM_KERNEL_TABULATED ? k.table : nullptr;
    return d;
}

}  // namespace sdm

extern "C" {

int sdm_abi_version(void) { return SDM_ABI_VERSION; }

const char *sdm_last_error(void) { return g_err; }

int sdm_create(sdm_ctx **ctx, int64_t n_sd_max, int32_t n_cell_max, int32_t n_attr_max)
{
    REQUIRE(ctx, "ctx is NULL");
    *ctx = nullptr;
    REQUIRE(n_sd_max >= 1 && n_sd_max <= ((int64_t)1 << 31), "n_sd_max out of range");
    REQUIRE(n_cell_max >= 1, "n_cell_max < 1");
    REQUIRE(n_attr_max >= 1 && n_attr_max <= 64, "n_attr_max out of range");
    sdm_ctx *c = nullptr;
    SDM_TRY
    c = new sdm_ctx();
    SDM_HIP(hipGetDevice(&c->device));
    c->n_sd_max = n_sd_max;
    c->n_cell_max = n_cell_max;
    c->n_attr_max = n_attr_max;
    const int64_t tiles = (n_sd_max + 2047) / 2048 + 2;
    hipError_t e = hipMalloc(&c->err_dev, 64);
    if (e == hipSuccess)
        e = hipMalloc(&c->tmp_u32, 4ull * (n_sd_max + 64));
    if (e == hipSuccess)
        e = hipMalloc(&c->tile_cnt, 4ull * (tiles + 1));
    if (e != hipSuccess) {
        destroy_ctx(c);
        return fail(e == hipErrorOutOfMemory ? SDM_E_NOMEM : SDM_E_HIP, "sdm_create: %s",
                    hipGetErrorString(e));
    }
    SDM_HIP(hipMemset(c->err_dev, 0, 64));
    SDM_HIP(hipDeviceSynchronize());
    *ctx = c;
    c = nullptr;
    }
    catch (const ::sdm::HipError &he)
    {
        destroy_ctx(c);
        return ::sdm::fail(SDM_E_HIP, "%s: %s", he.what, hipGetErrorString(he.e));
    }
    catch (...)
    {
        destroy_ctx(c);
        return ::sdm::fail(SDM_E_NOMEM, "sdm_create failed");
    }
    return SDM_OK;
}

int sdm_destroy(sdm_ctx *ctx)
{
    if (!ctx)
        return SDM_OK;
    (void)hipDeviceSynchronize();
    destroy_ctx(ctx);
    return SDM_OK;
}

int sdm_read_errors(sdm_ctx *ctx, uint32_t *flags)
{
    REQUIRE(ctx && flags, "null argument");
    SDM_TRY
    SDM_HIP(hipDeviceSynchronize());
    SDM_HIP(hipMemcpy(flags, ctx->err_dev, 4, hipMemcpyDeviceToHost));
    SDM_HIP(hipMemset(ctx->err_dev, 0, 4));
    SDM_HIP(hipDeviceSynchronize());
    SDM_CATCH
}

int sdm_set_plan_limits(sdm_ctx *ctx, int32_t bucket_target, int32_t group_cap)
{
    REQUIRE(ctx, "ctx is NULL");
    REQUIRE(bucket_target >= 0, "bucket_target < 0");
    SDM_TRY
    SDM_HIP(hipDeviceSynchronize());
    for (auto &kv : ctx->plans)
        free_plan(kv.second);
    ctx->plans.clear();
    ctx->dbg_bucket_target = bucket_target;
    ctx->dbg_group_cap = group_cap;
    SDM_CATCH
}

int sdm_prepare_step(sdm_ctx *ctx, const sdm_state *st, const sdm_step_params *p)
{
    if (int rc = check_state(ctx, st, p))
        return rc;
    SDM_TRY
    (void)get_plan(ctx, MODE_FUSED, st->n_sd, st->n_cell, p->expected_per_cell);
    SDM_CATCH
}

int sdm_step(sdm_ctx *ctx, const sdm_state *st, const sdm_step_params *p, hipStream_t stream)
{
    if (int rc = check_state(ctx, st, p))
        return rc;
    if (st->n_sd == 0)
        return SDM_OK;
    SDM_TRY
    Plan *plan = get_plan(ctx, MODE_FUSED, st->n_sd, st->n_cell, p->expected_per_cell);
    StepInputs in;
    in.n_sd = st->n_sd;
    in.xi = st->xi;
    in.attr = st->attr;
    in.n_attr = st->n_attr;
    in.stride = st->attr_stride;
    in.cell_id = st->cell_id;
    in.seed = p->rng.seed;
    in.run = p->rng.run;
    in.step = p->rng.step;
    in.step_dev = p->rng.step_dev;
    in.step_advance = p->step_advance;
    in.dt = p->dt;
    in.dv_cell = p->dv_per_cell;
    in.dv = p->dv;
    in.kern = kernel_desc(p->kernel);
    in.idx_out = st->idx;
    in.cell_start = st->cell_start;
    in.n_live_out = st->n_live_dev;
    in.counters = st->counters_dev;
    in.gamma_out = st->gamma_out;
    for (int i = 0; i < 4; ++i)
        in.events[i] = p->events[i];
    if (st->gamma_out && st->n_sd >= 2) {
        const int64_t n = st->n_sd / 2;
        hipLaunchKernelGGL(k_fill_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           stream, st->gamma_out, n);
    }
    engine_run(ctx, plan, in, stream);
    SDM_CATCH
}

}  // extern "C"

// ------------------------------------------------------------ batches
static uint64_t layout_key(const std::vector<sdm_segment> &segs)
{
    uint64_t h = 1469598103934665603ull;  // FNV-1a over (offset, n_sd)
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xFFu;
            h *= 1099511628211ull;
        }
    };
    mix(segs.size());
    for (const auto &g : segs) {
        mix((uint64_t)g.offset);
        mix((uint64_t)g.n_sd);
    }
    return h;
}

static int check_batch_state(const sdm_ctx *ctx, const sdm_batch *b, const sdm_state *st,
                             const sdm_step_params *p)
{
    REQUIRE(ctx && b && st && p, "null argument");
    REQUIRE(st->n_cell == (int32_t)b->segs.size(), "state n_cell != number of segments");
    REQUIRE(st->n_sd >= b->n_items && st->n_sd <= ctx->n_sd_max, "state n_sd too small");
    REQUIRE(st->n_attr >= 1 && st->n_attr <= ctx->n_attr_max, "n_attr out of range");
    REQUIRE(st->attr_stride >= st->n_sd, "attr_stride < n_sd");
    REQUIRE(st->xi && st->attr && st->idx && st->n_live_dev && st->cell_start,
            "state pointer is NULL");
    REQUIRE(((uintptr_t)st->xi & 15) == 0 && ((uintptr_t)st->attr & 15) == 0,
            "xi and attr must be 16-byte aligned");
    REQUIRE(std::isfinite(p->dt) && p->dt >= 0, "dt invalid");
    return SDM_OK;
}

static void batch_inputs(sdm_batch *b, const sdm_state *st, const sdm_step_params *p,
                         StepInputs &in)
{
    in.n_sd = b->n_items;
    in.xi = st->xi;
    in.attr = st->attr;
    in.n_attr = st->n_attr;
    in.stride = st->attr_stride;
    in.cell_id = nullptr;
    in.seed = p->rng.seed;
    in.run = 0;
    in.step = p->rng.step;
    in.step_dev = p->rng.step_dev;
    in.step_advance = p->step_advance;
    in.dt = p->dt;
    in.idx_out = st->idx;
    in.cell_start = st->cell_start;
    in.n_live_out = st->n_live_dev;
    in.counters = st->counters_dev;
    in.gamma_out = st->gamma_out;
    in.slot_cell_local = true;
    for (int i = 0; i < 4; ++i)
        in.events[i] = p->events[i];
}

extern "C" {

int sdm_batch_create(sdm_ctx *ctx, sdm_batch **b, const sdm_segment *segs, int32_t n_seg)
{
    REQUIRE(ctx && b && segs, "null argument");
    *b = nullptr;
    REQUIRE(n_seg >= 1 && n_seg <= ctx->n_cell_max, "n_seg out of range");
    int64_t end = 0;
    for (int32_t i = 0; i < n_seg; ++i) {
        const sdm_segment &g = segs[i];
        REQUIRE(g.offset >= end && (g.offset & 1) == 0, "segment %d: offset must be even and "
                "not overlap the previous segment", i);
        REQUIRE(g.n_sd >= 0 && g.offset + g.n_sd <= ctx->n_sd_max, "segment %d: size", i);
        REQUIRE(g.dv > 0 && std::isfinite(g.dv), "segment %d: dv", i);
        if (int rc = check_kernel(g.kernel, "segment kernel"))
            return rc;
        end = g.offset + g.n_sd;
    }
    sdm_batch *nb = nullptr;
    SDM_TRY
    nb = new sdm_batch();
    nb->segs.assign(segs, segs + n_seg);
    nb->n_items = end;
    nb->schedule = 0;
    nb->plan = build_batch_plan(ctx, nb->segs, nb->n_items, 0);
    *b = nb;
    nb = nullptr;
    }
    catch (const ::sdm::HipError &he)
    {
        delete nb;
        return ::sdm::fail(SDM_E_UNSUPPORTED, "%s: %s", he.what, hipGetErrorString(he.e));
    }
    catch (...)
    {
        delete nb;
        return ::sdm::fail(SDM_E_NOMEM, "sdm_batch_create failed");
    }
    return SDM_OK;
}

int sdm_batch_destroy(sdm_ctx *ctx, sdm_batch *b)
{
    (void)ctx;
    if (!b)
        return SDM_OK;
    (void)hipDeviceSynchronize();
    free_plan(b->plan);
    delete b;
    return SDM_OK;
}

int sdm_batch_step(sdm_ctx *ctx, sdm_batch *b, const sdm_state *st, const sdm_step_params *p,
                   hipStream_t stream)
{
    if (int rc = check_batch_state(ctx, b, st, p))
        return rc;
    SDM_TRY
    StepInputs in;
    batch_inputs(b, st, p, in);
    if (st->gamma_out && st->n_sd >= 2) {
        const int64_t n = st->n_sd / 2;
        hipLaunchKernelGGL(k_fill_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           stream, st->gamma_out, n);
    }
    engine_run(ctx, b->plan, in, stream);
    SDM_CATCH
}

int sdm_batch_set_schedule(sdm_ctx *ctx, sdm_batch *b, int32_t schedule, int32_t *n_sched)
{
    REQUIRE(ctx && b, "null argument");
    if (n_sched)
        *n_sched = n_schedules();
    if (schedule < 0)
        return SDM_OK;
    REQUIRE(schedule < n_schedules(), "schedule out of range");
    SDM_TRY
    if (schedule != b->schedule) {
        Plan *np = build_batch_plan(ctx, b->segs, b->n_items, schedule);
        SDM_HIP(hipDeviceSynchronize());
        free_plan(b->plan);
        b->plan = np;
        b->schedule = schedule;
    }
    SDM_CATCH
}

int sdm_autotune(sdm_ctx *ctx, sdm_batch *b, const sdm_state *scratch, const sdm_step_params *p,
                 int32_t steps, const char *cache_path, int32_t *chosen)
{
    if (int rc = check_batch_state(ctx, b, scratch, p))
        return rc;
    REQUIRE(steps >= 1, "steps < 1");
    const uint64_t key = layout_key(b->segs);
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SDM_TRY
    int best = -1;
    if (cache_path) {
        std::ifstream f(cache_path);
        std::string line;
        while (std::getline(f, line)) {
            std::istringstream ls(line);
            unsigned long long k = 0;
            int sch = -1;
            if ((ls >> std::hex >> k >> std::dec >> sch) && k == key && sch >= 0 &&
                sch < n_schedules())
                best = sch;
        }
    }
    if (best < 0) {
        SDM_HIP(hipStreamCreate(&s));
        SDM_HIP(hipEventCreate(&e0));
        SDM_HIP(hipEventCreate(&e1));
        // the distinct candidate plans, all kept until the choice is made
        std::vector<std::pair<int, Plan *>> cands;
        std::vector<::sdm::PlanShape> shapes;
        try {
            for (int sch = 0; sch < n_schedules(); ++sch) {
                Plan *cand = nullptr;
                try {
                    cand = build_batch_plan(ctx, b->segs, b->n_items, sch);
                } catch (const ::sdm::HipError &) {
                    continue;  // this schedule does not fit the plan limits
                }
                const ::sdm::PlanShape sh = ::sdm::shape_of(cand);
                if (std::find(shapes.begin(), shapes.end(), sh) != shapes.end()) {
                    free_plan(cand);  // the same plan as a schedule already listed
                    continue;
                }
                shapes.push_back(sh);
                cands.emplace_back(sch, cand);
            }
            // two passes, the second in reverse order, each candidate a
            // warm-up step and `steps` timed steps; a candidate's time is the
            // faster of its two (candidates are often within a few per cent
            // of each other, and the first steps on fresh allocations run
            // slow)
            std::vector<float> ms(cands.size(), 3.0e38f);
            StepInputs in;
            batch_inputs(b, scratch, p, in);
            in.gamma_out = nullptr;
            in.step_advance = nullptr;
            for (int i = 0; i < 4; ++i)
                in.events[i] = nullptr;
            uint32_t t_step = p->rng.step + 1u;
            for (int pass = 0; pass < 2; ++pass) {
                for (size_t k = 0; k < cands.size(); ++k) {
                    const size_t c = pass == 0 ? k : cands.size() - 1 - k;
                    in.step = t_step++;
                    engine_run(ctx, cands[c].second, in, s);  // warm-up
                    SDM_HIP(hipEventRecord(e0, s));
                    for (int t = 0; t < steps; ++t) {
                        in.step = t_step++;
                        engine_run(ctx, cands[c].second, in, s);
                    }
                    SDM_HIP(hipEventRecord(e1, s));
                    SDM_HIP(hipEventSynchronize(e1));
                    float rep_ms = 0.f;
                    SDM_HIP(hipEventElapsedTime(&rep_ms, e0, e1));
                    ms[c] = std::min(ms[c], rep_ms);
                }
            }
            size_t bi = 0;
            for (size_t c = 1; c < cands.size(); ++c)
                if (ms[c] < ms[bi])
                    bi = c;
            if (!cands.empty())
                best = cands[bi].first;
        } catch (...) {
            for (auto &c : cands)
                free_plan(c.second);
            throw;
        }
        for (auto &c : cands)
            free_plan(c.second);
        if (best < 0)
            throw ::sdm::HipError{hipErrorInvalidValue, "no schedule fits this batch"};
        if (cache_path) {
            std::ofstream f(cache_path, std::ios::app);
            f << std::hex << (unsigned long long)key << std::dec << " " << best << "\n";
        }
    }
    if (best != b->schedule) {
        Plan *np = build_batch_plan(ctx, b->segs, b->n_items, best);
        SDM_HIP(hipDeviceSynchronize());
        free_plan(b->plan);
        b->plan = np;
        b->schedule = best;
    }
    if (chosen)
        *chosen = best;
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (s)
        (void)hipStreamDestroy(s);
    }
    catch (const ::sdm::HipError &he)
    {
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        if (s)
            (void)hipStreamDestroy(s);
        return ::sdm::fail(SDM_E_HIP, "%s: %s", he.what, hipGetErrorString(he.e));
    }
    catch (...)
    {
        return ::sdm::fail(SDM_E_STATE, "sdm_autotune failed");
    }
    return SDM_OK;
}

}  // extern "C"
