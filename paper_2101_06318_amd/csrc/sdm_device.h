// Device-side building blocks of the SDM coagulation step on gfx950:
// counter-based uniforms, coalescence kernels and the pairwise collision
// update.  Definitions follow arXiv:2101.06318 (eqs. 3-6) and the uniform
// stream described in include/sdm.h.  Compiled with -ffp-contract=off so
// every floating-point operation below is one IEEE binary64 operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdm {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11).  With a wave-uniform key the round
// keys live in scalar registers; each round is two 32x32->64 multiplies.
struct Block4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Block4 philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                         uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block4{c0, c1, c2, c3};
}

// 64-bit words of elements 2m (lo) and 2m+1 (hi) of a stream.
struct WordPair {
    uint64_t even, odd;
};

__device__ __forceinline__ WordPair philox_words(uint64_t seed, uint32_t run,
                                                 uint32_t step, uint32_t stream,
                                                 uint64_t pair_index)
{
    const Block4 b = philox((uint32_t)pair_index, step, stream, run,
                            (uint32_t)seed, (uint32_t)(seed >> 32));
    return WordPair{((uint64_t)b.w0 << 32) | b.w1, ((uint64_t)b.w2 << 32) | b.w3};
}

__device__ __forceinline__ uint64_t philox_word(uint64_t seed, uint32_t run,
                                                uint32_t step, uint32_t stream,
                                                uint64_t e)
{
    const WordPair w = philox_words(seed, run, step, stream, e >> 1);
    return (e & 1) ? w.odd : w.even;
}

// 53-bit uniform in [0, 1) from a Philox word.
__device__ __forceinline__ double word_to_uniform(uint64_t w)
{
    return (double)(w >> 11) * 0x1p-53;
}

// Sort key of a given uniform: floor(u * 2^53); values outside [0, 1)
// (and NaN) are clamped into the key range.
__device__ __forceinline__ uint64_t uniform_to_key(double u)
{
    if (!(u > 0.0))
        return 0;
    if (u >= 1.0)
        return (1ull << 53) - 1;
    return (uint64_t)(u * 9007199254740992.0);
}

// ------------------------------------------------------------- kernels
enum { KERNEL_GOLOVIN = 0, KERNEL_GEOMETRIC = 1, KERNEL_CONSTANT = 2,
       KERNEL_MULTIPLICATIVE = 3, KERNEL_TABULATED = 4 };

struct KernelDesc {
    int32_t id;
    int32_t reserved;
    double p[4];
    const double *table;  // KERNEL_TABULATED: n x n, row-major
};

// Cell of volume v in a tabulated kernel: the IEEE pattern of v shifted
// right by 52 - m, less lo, clamped to [0, n - 1] (integer operations only).
__device__ __forceinline__ int64_t table_cell(double v, int64_t lo, int64_t n, int m)
{
    const int64_t c = (int64_t)((uint64_t)__double_as_longlong(v) >> (52 - m)) - lo;
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

#define SDM_PI_D 3.141592653589793

// Cube root by Newton's iteration y <- (2y + x/y^2)/3 from the power of two
// nearest below x^(1/3); 8 steps reach full binary64 precision over the
// normal range.  Only +, *, / and exact scalings, so host and device agree
// bit for bit.
__device__ __forceinline__ double cbrt_newton(double x)
{
    if (x == 0.0)
        return 0.0;
    int e;
    (void)frexp(x, &e);
    int q = e / 3;
    if (e % 3 < 0)
        q -= 1;
    double y = ldexp(1.0, q);
#pragma unroll
    for (int it = 0; it < 8; ++it)
        y = (2.0 * y + x / (y * y)) / 3.0;
    return y;
}

// Terminal velocity [m/s] of a drop of radius r [m]: three power laws,
// k1 r^2, k2 r and k3 sqrt(r) (k1 = 1.19e8 1/(m s), k2 = 8e3 1/s,
// k3 = 201 m^0.5/s), each used up to the radius where it meets the next one
// (k2/k1 = 67.2 um and (k3/k2)^2 = 631 um), so that w is continuous.
constexpr double VT_K1 = 1.19e8;
constexpr double VT_K2 = 8.0e3;
constexpr double VT_K3 = 201.0;

__device__ __forceinline__ double terminal_velocity(double r)
{
    constexpr double r12 = VT_K2 / VT_K1;
    constexpr double r23 = (VT_K3 / VT_K2) * (VT_K3 / VT_K2);
    if (r < r12)
        return VT_K1 * (r * r);
    if (r < r23)
        return VT_K2 * r;
    return VT_K3 * sqrt(r);
}

__device__ __forceinline__ double kernel_value(const KernelDesc &k, double v1,
                                               double v2)
{
    switch (k.id) {
    case KERNEL_GOLOVIN:
        return k.p[0] * (v1 + v2);
    case KERNEL_GEOMETRIC: {
        const double r1 = cbrt_newton((0.75 * v1) / SDM_PI_D);
        const double r2 = cbrt_newton((0.75 * v2) / SDM_PI_D);
        const double w1 = terminal_velocity(r1);
        const double w2 = terminal_velocity(r2);
        const double rs = r1 + r2;
        return ((SDM_PI_D * (rs * rs)) * fabs(w1 - w2)) * k.p[0];
    }
    case KERNEL_CONSTANT:
        return k.p[0];
    case KERNEL_MULTIPLICATIVE:
        return k.p[0] * (v1 * v2);
    case KERNEL_TABULATED: {
        const int64_t lo = (int64_t)k.p[1], n = (int64_t)k.p[2];
        const int m = (int)k.p[3];
        const int64_t i1 = table_cell(v1, lo, n, m), i2 = table_cell(v2, lo, n, m);
        const int64_t a = i1 < i2 ? i1 : i2, b = i1 < i2 ? i2 : i1;
        return k.p[0] * k.table[a * n + b];
    }
    default:
        return 0.0;
    }
}

// ------------------------------------------------- pair-rate upper bounds
// A pair collides only if its gamma = ceil(p - phi) is at least 1, i.e. only
// if p > phi.  With nonnegative factors, p >= 0 and phi < 1, so a pair whose
// upper bound P >= p is below phi has p - phi in (-1, 0) and gamma = -0.0
// exactly: no collision, nothing to read or write.  The bound is built from
// per-SD codes that the tile kernel packs into each record:
//  * volume code (13 bits): the IEEE pattern of v >= 0 read as an integer is
//    monotone in v; rounded up to a multiple of 2^50 (two mantissa bits
//    kept) it decodes to a double in [v, 1.25 v].  +inf, NaN and negative v
//    (sign bit set) give codes that decode to +inf or NaN;
//  * multiplicity code (8 bits): the same on (double)xi, relative to 1.0;
//    255 decodes to +inf.
// P evaluates each kernel in its own operation order with the decoded
// bounds (every step is monotone for nonnegative operands under round to
// nearest), times 1 + 2^-9, which also covers the gravitational kernel's
// cube root and terminal velocity taken in single precision there.  A NaN
// or infinite P never rules a pair out.
constexpr uint32_t VCODE_INF = 8191u;
constexpr uint32_t XCODE_INF = 255u;

__device__ __forceinline__ uint32_t vcode_up(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    if (u >= 0x7FF0000000000000ull)  // +inf, NaN, negative (and -0.0)
        return VCODE_INF;
    return (uint32_t)((u + ((1ull << 50) - 1ull)) >> 50);
}

__device__ __forceinline__ double vcode_decode(uint32_t c)
{
    return __longlong_as_double((long long)((uint64_t)c << 50));
}

__device__ __forceinline__ uint32_t xcode_up(uint64_t xi)  // xi >= 1
{
    const uint64_t u = (uint64_t)__double_as_longlong((double)xi) - 0x3FF0000000000000ull;
    const uint64_t c = (u + ((1ull << 50) - 1ull)) >> 50;
    return c < XCODE_INF ? (uint32_t)c : XCODE_INF;
}

__device__ __forceinline__ double xcode_decode(uint32_t c)
{
    return c >= XCODE_INF ? __longlong_as_double(0x7FF0000000000000ll)
                          : __longlong_as_double((long long)(0x3FF0000000000000ull +
                                                             ((uint64_t)c << 50)));
}

// Upper bound of cbrt(x) for x >= 0: x rounded up to single precision
// (normal range), cube root as exp2(log2(x)/3) in single precision (error
// below 1e-5 relative), then raised by 2^-10.
__device__ __forceinline__ double cbrt_upper(double x)
{
    if (!(x > 0.0))
        return x == 0.0 ? 0.0 : x;  // 0, or NaN propagates
    if (!(x < 3.0e38))
        return __longlong_as_double(0x7FF0000000000000ll);  // beyond float: no bound
    float xf = (float)x;
    if ((double)xf < x)
        xf = __uint_as_float(__float_as_uint(xf) + 1u);
    xf = fmaxf(xf, 1.17549435e-38f);
    const float y = exp2f(log2f(xf) * (1.0f / 3.0f));
    return (double)y * (1.0 + 0x1p-10);
}

__device__ __forceinline__ double kernel_bound(int32_t kid, double kp, double V1, double V2)
{
    switch (kid) {
    case KERNEL_GOLOVIN:
        return kp * (V1 + V2);
    case KERNEL_GEOMETRIC: {
        const double R1 = cbrt_upper((0.75 * V1) / SDM_PI_D);
        const double R2 = cbrt_upper((0.75 * V2) / SDM_PI_D);
        const double W = fmax(terminal_velocity(R1), terminal_velocity(R2));
        const double rs = R1 + R2;
        return ((SDM_PI_D * (rs * rs)) * W) * kp;
    }
    case KERNEL_CONSTANT:
        return kp;
    case KERNEL_MULTIPLICATIVE:
        return kp * (V1 * V2);
    default:
        return __longlong_as_double(0x7FF8000000000000ll);
    }
}

// Codes of one SD as the record carries them: xi code | volume code << 8.
__device__ __forceinline__ uint32_t sd_codes(uint64_t xi, double v)
{
    return xcode_up(xi) | (vcode_up(v) << 8);
}

// F(n) = ((n^2 - n)/2) / floor(n/2): n - 1 for even n, n for odd n.
__device__ __forceinline__ uint64_t pair_scale(uint64_t n)
{
    if (n < 2)
        return 0;
    return (n & 1) ? n : n - 1;
}

// Rate gamma as a count: NaN, negatives and -0.0 read as 0; >= 2^64 saturates.
__device__ __forceinline__ uint64_t gamma_count(double g)
{
    if (!(g >= 1.0))
        return 0;
    if (g >= 18446744073709551616.0)
        return ~0ull;
    return (uint64_t)g;
}

// Collision statistics gathered per thread, reduced per workgroup.
struct Stats {
    uint32_t pairs, coll, capped, zeroed, ge2;
};

// Outcome of eqs. (4)-(6) for one pair.  (a, b) are the SDs at the opening
// and the following sorted positions.  Returns g (gamma-tilde); on g > 0 it
// fills the new multiplicities and tells which SD is j (the larger).
struct Collision {
    uint64_t g;
    uint64_t xj_new, xk_new;
    bool a_is_j;
    bool split;  // case 2 (equal-multiplicity split)
};

__device__ __forceinline__ Collision collide(uint64_t xa, uint64_t xb, double gamma,
                                             Stats &st)
{
    Collision c;
    c.a_is_j = !(xa < xb);
    const uint64_t xj = c.a_is_j ? xa : xb;
    const uint64_t xk = c.a_is_j ? xb : xa;
    st.pairs += 1;
    c.g = 0;
    c.split = false;
    c.xj_new = xj;
    c.xk_new = xk;
    if (xk == 0)
        return c;
    const uint64_t G = gamma_count(gamma);
    if (G == 0)
        return c;
    // g = min(G, floor(xj/xk)); the 64-bit division is only needed when
    // G >= 2, since xj >= xk makes floor(xj/xk) >= 1.
    uint64_t g = 1;
    if (G >= 2) {
        st.ge2 += 1;
        const uint64_t ratio = xj / xk;
        g = G < ratio ? G : ratio;
        if (g < G)
            st.capped += 1;
    }
    st.coll += 1;
    c.g = g;
    const uint64_t d = xj - g * xk;
    if (d > 0) {
        c.xj_new = d;
    } else {
        const uint64_t h = xk / 2;
        c.xj_new = h;
        c.xk_new = xk - h;
        c.split = true;
        if (h == 0)
            st.zeroed += 1;
    }
    return c;
}

// Attribute update for one attribute row: eq. (5) adds g A_j to A_k; in
// eq. (6) both SDs take that sum.
__device__ __forceinline__ void collide_attr(double &Aj, double &Ak, uint64_t g,
                                             bool split)
{
    const double merged = Ak + (double)g * Aj;
    Ak = merged;
    if (split)
        Aj = merged;
}

// Attribute rows r0 .. n_attr - 1 of a colliding pair.
__device__ __forceinline__ void collide_rows(double *attr, int r0, int n_attr, int64_t stride,
                                             uint32_t sj, uint32_t sk, uint64_t g, bool split)
{
    for (int r = r0; r < n_attr; ++r) {
        double *A = attr + (int64_t)r * stride;
        double Aj = A[sj], Ak = A[sk];
        collide_attr(Aj, Ak, g, split);
        A[sj] = Aj;
        A[sk] = Ak;
    }
}

// Writes the outcome of a pair with g > 0 to the global state.
__device__ __forceinline__ void apply_collision(const Collision &c, uint32_t sa,
                                                uint32_t sb, uint64_t *xi,
                                                double *attr, int n_attr,
                                                int64_t stride)
{
    const uint32_t sj = c.a_is_j ? sa : sb;
    const uint32_t sk = c.a_is_j ? sb : sa;
    xi[sj] = c.xj_new;
    xi[sk] = c.xk_new;
    collide_rows(attr, 0, n_attr, stride, sj, sk, c.g, c.split);
}

// apply_collision for a caller that holds the pair's volumes (attribute
// row 0) already: row 0 is written without reading it back.
__device__ __forceinline__ void apply_collision_v(const Collision &c, uint32_t sa,
                                                  uint32_t sb, double va, double vb,
                                                  uint64_t *xi, double *attr, int n_attr,
                                                  int64_t stride)
{
    const uint32_t sj = c.a_is_j ? sa : sb;
    const uint32_t sk = c.a_is_j ? sb : sa;
    xi[sj] = c.xj_new;
    xi[sk] = c.xk_new;
    double Vj = c.a_is_j ? va : vb, Vk = c.a_is_j ? vb : va;
    collide_attr(Vj, Vk, c.g, c.split);
    attr[sj] = Vj;
    attr[sk] = Vk;
    if (n_attr > 1)
        collide_rows(attr, 1, n_attr, stride, sj, sk, c.g, c.split);
}

// Inclusive scan over the 64 lanes of a wave on DPP operands (no LDS trip):
// Hillis-Steele within each 16-lane row (shifts by 1, 2, 4, 8; lanes with no
// source add 0), then the last lane of row 0 into row 1 and of row 2 into
// row 3, then the last lane of row 1 into rows 2 and 3.  Every lane of the
// wave must be active.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xF, true);
}

__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t v)
{
    v += dpp_lane<0x111, 0xF>(v);  // row_shr:1
    v += dpp_lane<0x112, 0xF>(v);  // row_shr:2
    v += dpp_lane<0x114, 0xF>(v);  // row_shr:4
    v += dpp_lane<0x118, 0xF>(v);  // row_shr:8
    v += dpp_lane<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_lane<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Workgroup reduction of the statistics into counters[8] (one atomic per
// nonzero slot per workgroup).  `red` is LDS scratch of 5*(threads/64) words.
template <int THREADS>
__device__ __forceinline__ void flush_stats(const Stats &st, uint64_t *counters,
                                            uint32_t *red)
{
    constexpr int W = THREADS / 64;
    uint32_t v[5] = {st.pairs, st.coll, st.capped, st.zeroed, st.ge2};
#pragma unroll
    for (int i = 0; i < 5; ++i)
        v[i] = wave_scan_u32(v[i]);  // lane 63: the wave's sum
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
            red[i * W + wid] = v[i];
    }
    __syncthreads();
    if (threadIdx.x < 5 && counters) {
        uint64_t s = 0;
        for (int w = 0; w < W; ++w)
            s += red[threadIdx.x * W + w];
        if (s)
            atomicAdd((unsigned long long *)&counters[threadIdx.x],
                      (unsigned long long)s);
    }
}

__device__ __forceinline__ uint32_t step_of(uint32_t step, const uint32_t *step_dev)
{
    return step_dev ? *step_dev : step;
}

}  // namespace sdm
