// Context management, error reporting and the fused timestep entry points
// of the C ABI (include/sdm.h).
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <new>

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
    REQUIRE(st->xi && st->attr && st->idx && st->n_live_dev && st->cell_start,
            "state pointer is NULL");
    REQUIRE(st->n_cell == 1 || st->cell_id, "cell_id is NULL with n_cell > 1");
    REQUIRE(((uintptr_t)st->xi & 15) == 0, "xi must be 16-byte aligned");
    REQUIRE(p->dv_per_cell || p->dv > 0, "need dv_per_cell or dv > 0");
    REQUIRE(p->kernel.id >= SDM_KERNEL_GOLOVIN && p->kernel.id <= SDM_KERNEL_MULTIPLICATIVE,
            "unknown kernel id %d", p->kernel.id);
    REQUIRE(std::isfinite(p->dt) && p->dt >= 0, "dt invalid");
    return SDM_OK;
}

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
    in.kern.id = p->kernel.id;
    for (int i = 0; i < 4; ++i)
        in.kern.p[i] = p->kernel.p[i];
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
