// Moment-surrogate network on the gfx950 matrix cores.
//
// The network (5 -> 128 -> 128 -> 128 -> 3, GELU) is small enough that a
// whole forward or backward pass of a 16-sample tile stays in one wave's
// registers.  Every matmul is v_mfma_f32_16x16x32_bf16 in transposed form,
// Z^T = W A^T: the weights are the M x K operand and the activations of 16
// samples the K x N operand.  The 16x16 result of one output tile leaves
// lane (r, g) = (lane % 16, lane / 16) holding neurons 16t + 4g + e
// (e = 0..3) of sample r, which is almost the layout the next matmul needs
// for its K x N operand (lane (r, g) holding 8 consecutive K slots
// 8g..8g+7 of sample r).  Since the contraction may visit K in any order,
// the K slots of K-step q are mapped to neurons by
//   slot 8g + e  ->  32q + 4g + e        (e < 4, from output tile 2q)
//   slot 8g + e  ->  32q + 16 + 4g + e-4 (e >= 4, from output tile 2q+1)
// and the weights are stored ("packed") with the same permutation, so the
// activations never leave the registers between layers.
//
// Batches of up to a few tiles per SIMD use a variant in which four waves
// share a tile's hidden layers (k_mlp_forward_split), which spreads the
// GELU work over more waves.
//
// Training: the forward pass also keeps, per hidden unit, GELU'(z) and the
// bf16 activation it fed to the next layer, so the backward pass is matmuls
// and products only.  Weight gradients dW = dZ^T A sum over samples, a
// different operand layout; there the workgroup stages dZ^T and A^T of its
// 64 samples in LDS and each wave takes a share of the output tiles.
// Per-workgroup partial sums are reduced in a fixed order by a second kernel
// (deterministic).
#include <math.h>

#include <cmath>

#include "sdm_internal.h"

using namespace sdm;

namespace {

constexpr int NIN = 5, NH = 128, NOUT = 3;
constexpr int OFF_W1 = 0, OFF_B1 = 640, OFF_W2 = 768, OFF_B2 = 17152, OFF_W3 = 17280,
              OFF_B3 = 33664, OFF_W4 = 33792, OFF_B4 = 34176, NPARAM = 34179;
static_assert(NPARAM == SDM_MLP_N_PARAMS, "parameter count");

// Packed fragments: 64 lanes x 8 bf16 (1 KiB) each.
//   F1 [t]     layer 1, K = 5 input features padded to 32 (natural order)
//   F2 [t][q]  layer 2 (permuted K)      F3 [t][q] layer 3
//   F4 [q]     layer 4, M = 3 outputs padded to 16
//   B4 [t]     W4^T for dH3 = W4^T dZ4 (K = 3 padded to 32, natural order)
//   B3 [t][q]  W3^T for dH2               B2 [t][q] W2^T for dH1
constexpr int FR_F1 = 0, FR_F2 = 8, FR_F3 = 40, FR_F4 = 72, FR_B4 = 76, FR_B3 = 84,
              FR_B2 = 116, FR_N = 148, FWD_FRAGS = 76;
static_assert(FR_N * 1024 == SDM_MLP_PACKED_BYTES, "packed size");
// Training cache of a 16-sample tile: GELU'(z) of the three hidden layers
// (fp32, [layer][t][lane] f32x4, the MFMA output layout) and the bf16
// activations GELU(z) the forward pass fed to the next layer ([layer][t][lane]
// two words), so that the backward pass evaluates no transcendental.
constexpr int CACHE_GG = 3 * 8 * 64 * 4;       // floats
constexpr int CACHE_TILE = CACHE_GG + 3 * 8 * 64 * 2;
static_assert(CACHE_TILE == 16 * SDM_MLP_CACHE_FLOATS_PER_ROW, "cache tile size");

constexpr int BWD_CHUNK = 64;      // samples per backward workgroup pass
constexpr int BWD_ROW = 72;        // LDS row stride (bf16): 64 samples + 8 pad
constexpr int PART_ROWS_MAX = 128; // backward workgroups (partial-sum rows)
constexpr int FWD_GRID_MAX = 512;  // forward workgroups (two per CU)
constexpr int64_t SPLIT_MAX_TILES = 16384;  // largest batch (16-sample tiles) for the split forward

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

__device__ inline f32x4 mfma(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// float -> bfloat16 bits, round to nearest even (finite inputs).
__device__ inline uint32_t bf16_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ inline uint32_t pack2(float lo, float hi)
{
    return bf16_bits(lo) | (bf16_bits(hi) << 16);
}

__device__ inline float gelu(float z)
{
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

// gelu(z) (the same expression, so the same bits) and its derivative
// Phi(z) + z phi(z), with one erf.
__device__ inline void gelu_both(float z, float &h, float &gg)
{
    const float e = erff(z * 0.70710678118654752f);
    h = 0.5f * z * (1.0f + e);
    gg = 0.5f * (1.0f + e) + z * (expf(-0.5f * z * z) * 0.39894228040143268f);
}

__device__ inline float *cache_gg(float *cache, int64_t tile, int layer, int t, int lane)
{
    return cache + tile * CACHE_TILE + ((layer * 8 + t) * 64 + lane) * 4;
}

__device__ inline uint32_t *cache_h(float *cache, int64_t tile, int layer, int t, int lane)
{
    return reinterpret_cast<uint32_t *>(cache + tile * CACHE_TILE + CACHE_GG +
                                        ((layer * 8 + t) * 64 + lane) * 2);
}

// Epilogue of one output tile (4 neurons of a lane): the bf16 activations as
// two words, and in training the cache entries.
template <bool TRAIN>
__device__ inline void gelu_tile(const f32x4 &z, uint32_t &w0, uint32_t &w1,
                                 float *__restrict__ cache, int64_t tile, bool tv, int layer,
                                 int t, int lane)
{
    float h[4];
    if (TRAIN) {
        float g4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            gelu_both(z[e], h[e], g4[e]);
        const f32x4 gg{g4[0], g4[1], g4[2], g4[3]};
        w0 = pack2(h[0], h[1]);
        w1 = pack2(h[2], h[3]);
        if (tv) {
            *(f32x4 *)cache_gg(cache, tile, layer, t, lane) = gg;
            *(uint2 *)cache_h(cache, tile, layer, t, lane) = make_uint2(w0, w1);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            h[e] = gelu(z[e]);
        w0 = pack2(h[0], h[1]);
        w1 = pack2(h[2], h[3]);
    }
}

__device__ inline int perm32(int p)
{
    const int g = p >> 3, e = p & 7;
    return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4);
}

// Master weight behind packed bf16 element i (0 for padding).
__device__ inline float pack_source(const float *P, int i)
{
    const int f = i >> 9, l = (i >> 3) & 63, e = i & 7;
    const int r = l & 15, p = 8 * (l >> 4) + e;
    if (f < FR_F2)
        return p < NIN ? P[OFF_W1 + (16 * f + r) * NIN + p] : 0.0f;
    if (f < FR_F3) {
        const int t = (f - FR_F2) >> 2, q = (f - FR_F2) & 3;
        return P[OFF_W2 + (16 * t + r) * NH + 32 * q + perm32(p)];
    }
    if (f < FR_F4) {
        const int t = (f - FR_F3) >> 2, q = (f - FR_F3) & 3;
        return P[OFF_W3 + (16 * t + r) * NH + 32 * q + perm32(p)];
    }
    if (f < FR_B4) {
        const int q = f - FR_F4;
        return r < NOUT ? P[OFF_W4 + r * NH + 32 * q + perm32(p)] : 0.0f;
    }
    if (f < FR_B3)
        return p < NOUT ? P[OFF_W4 + p * NH + 16 * (f - FR_B4) + r] : 0.0f;
    if (f < FR_B2) {
        const int t = (f - FR_B3) >> 2, q = (f - FR_B3) & 3;
        return P[OFF_W3 + (32 * q + perm32(p)) * NH + 16 * t + r];
    }
    const int t = (f - FR_B2) >> 2, q = (f - FR_B2) & 3;
    return P[OFF_W2 + (32 * q + perm32(p)) * NH + 16 * t + r];
}

__global__ void k_mlp_pack(uint32_t *__restrict__ packed, const float *__restrict__ P)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;  // one 32-bit word = 2 bf16
    if (w < FR_N * 256)
        packed[w] = pack2(pack_source(P, 2 * w), pack_source(P, 2 * w + 1));
}

// Bias, GELU and bf16 rounding of output tile t of a hidden layer; the
// rounded activations go to K-step t/2 of the next layer's operand.
template <int S, bool TRAIN>
__device__ inline void hidden_epilogue(const f32x4 (&acc)[S], int t, int layer,
                                       const float *__restrict__ sb, u32x4 (&out)[S][4],
                                       float *__restrict__ cache, int64_t tile0, int64_t n_tiles,
                                       int lane)
{
    const int g = lane >> 4;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        f32x4 z;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            z[e] = acc[j][e] + sb[layer * NH + 16 * t + 4 * g + e];
        uint32_t w0, w1;
        gelu_tile<TRAIN>(z, w0, w1, cache, tile0 + j, tile0 + j < n_tiles, layer, t, lane);
        const int q = t >> 1;
        if (t & 1) {
            out[j][q][2] = w0;
            out[j][q][3] = w1;
        } else {
            out[j][q][0] = w0;
            out[j][q][1] = w1;
        }
    }
}

template <int S, bool TRAIN>
__device__ inline void hidden_layer(const u32x4 *__restrict__ frags, int layer,
                                    const float *__restrict__ sb, const u32x4 (&in)[S][4],
                                    u32x4 (&out)[S][4], float *__restrict__ cache, int64_t tile0,
                                    int64_t n_tiles, int lane)
{
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        f32x4 acc[S];
#pragma unroll
        for (int j = 0; j < S; ++j)
            acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32x4 a = frags[(t * 4 + q) * 64 + lane];
#pragma unroll
            for (int j = 0; j < S; ++j)
                acc[j] = mfma(a, in[j][q], acc[j]);
        }
        hidden_epilogue<S, TRAIN>(acc, t, layer, sb, out, cache, tile0, n_tiles, lane);
        // one output tile's fragments at a time: left free, the scheduler
        // hoists the LDS reads of all eight tiles and the kernel spills
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int S, bool TRAIN>
__device__ inline void forward_tiles(float *__restrict__ y, float *__restrict__ cache,
                                     const float *__restrict__ x, int64_t B,
                                     const u32x4 *__restrict__ sw, const float *__restrict__ sb,
                                     int64_t tile0, int64_t n_tiles, int lane, int r, int g)
{
    u32x4 ha[S][4], hb[S][4];
    // layer 1: the K x N operand is x itself (features 8g..8g+7 of sample r)
    u32x4 bx[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int64_t s = (tile0 + j) * 16 + r;
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * g + e;
            v[e] = (k < NIN && s < B) ? x[s * NIN + k] : 0.0f;
        }
        bx[j] = u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const u32x4 a = sw[(FR_F1 + t) * 64 + lane];
        f32x4 acc[S];
#pragma unroll
        for (int j = 0; j < S; ++j)
            acc[j] = mfma(a, bx[j], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        hidden_epilogue<S, TRAIN>(acc, t, 0, sb, ha, cache, tile0, n_tiles, lane);
        __builtin_amdgcn_sched_barrier(0);
    }
    hidden_layer<S, TRAIN>(sw + FR_F2 * 64, 1, sb, ha, hb, cache, tile0, n_tiles, lane);
    hidden_layer<S, TRAIN>(sw + FR_F3 * 64, 2, sb, hb, ha, cache, tile0, n_tiles, lane);
    // layer 4: rows 0..2 of the 16-row output tile are the outputs
    f32x4 acc[S];
#pragma unroll
    for (int j = 0; j < S; ++j)
        acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const u32x4 a = sw[(FR_F4 + q) * 64 + lane];
#pragma unroll
        for (int j = 0; j < S; ++j)
            acc[j] = mfma(a, ha[j][q], acc[j]);
    }
    if (g == 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int64_t s = (tile0 + j) * 16 + r;
            if (s < B) {
#pragma unroll
                for (int e = 0; e < NOUT; ++e)
                    y[s * NOUT + e] = acc[j][e] + sb[3 * NH + e];
            }
        }
    }
}

// Forward pass.  Workgroup: 4 waves; each wave takes S consecutive
// 16-sample tiles at a time, striding over the batch (persistent grid), so
// the forward fragments (76 KiB) and biases are staged in LDS once per
// workgroup.
template <int S, bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_forward(float *__restrict__ y,
                                                     float *__restrict__ cache,
                                                     const float *__restrict__ x, int64_t B,
                                                     const u32x4 *__restrict__ packed,
                                                     const float *__restrict__ P)
{
    __shared__ u32x4 sw[FWD_FRAGS * 64];
    __shared__ float sb[3 * NH + 4];
    // staged with all of a thread's loads in flight together, then written
    // to LDS
    constexpr int NF = FWD_FRAGS * 64;
    constexpr int PER = NF / 256;
    static_assert(NF % 256 == 0, "fragments per thread");
    {
        u32x4 r[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j)
            r[j] = packed[threadIdx.x + 256 * j];
#pragma unroll
        for (int j = 0; j < PER; ++j)
            sw[threadIdx.x + 256 * j] = r[j];
    }
    for (int i = threadIdx.x; i < 3 * NH + NOUT; i += 256)
        sb[i] = P[i < NH ? OFF_B1 + i
                  : i < 2 * NH ? OFF_B2 + (i - NH)
                  : i < 3 * NH ? OFF_B3 + (i - 2 * NH)
                               : OFF_B4 + (i - 3 * NH)];
    __syncthreads();

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    const int64_t n_tiles = (B + 15) / 16;
    const int64_t stride = (int64_t)gridDim.x * 4 * S;
    for (int64_t tile0 = ((int64_t)blockIdx.x * 4 + w) * S; tile0 < n_tiles; tile0 += stride)
        forward_tiles<S, TRAIN>(y, cache, x, B, sw, sb, tile0, n_tiles, lane, r, g);
}


// Forward pass for batches that leave every SIMD about one 16-sample tile.
// A workgroup of 16 waves takes 4 tiles, and the 4 waves of a tile share
// each hidden layer: wave f computes output tiles 2f and 2f + 1, which make
// up K-step f of the next layer's operand, and the waves swap their K-steps
// through LDS.  The GELU work of a tile then runs on four waves that
// interleave on the SIMDs instead of one.
constexpr int SPLIT_TILES = 4;

template <bool TRAIN>
__device__ inline u32x4 split_epilogue(const f32x4 &a0, const f32x4 &a1, int t0, int layer,
                                       const float *__restrict__ sb, int g,
                                       float *__restrict__ cache, int64_t tile, bool tv, int lane)
{
    f32x4 z0, z1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        z0[e] = a0[e] + sb[layer * NH + 16 * t0 + 4 * g + e];
        z1[e] = a1[e] + sb[layer * NH + 16 * (t0 + 1) + 4 * g + e];
    }
    uint32_t w[4];
    gelu_tile<TRAIN>(z0, w[0], w[1], cache, tile, tv, layer, t0, lane);
    gelu_tile<TRAIN>(z1, w[2], w[3], cache, tile, tv, layer, t0 + 1, lane);
    return u32x4{w[0], w[1], w[2], w[3]};
}

template <bool TRAIN>
__global__ __launch_bounds__(1024) void k_mlp_forward_split(float *__restrict__ y,
                                                           float *__restrict__ cache,
                                                           const float *__restrict__ x,
                                                           int64_t B,
                                                           const u32x4 *__restrict__ packed,
                                                           const float *__restrict__ P)
{
    __shared__ u32x4 sw[FWD_FRAGS * 64];
    __shared__ float sb[3 * NH + 4];
    // K-steps of the three hidden layers' outputs, one buffer per layer, so
    // that a layer's writes never meet the reads of the layer before
    __shared__ u32x4 xk[3][SPLIT_TILES][4][64];
    constexpr int NF = FWD_FRAGS * 64;
    constexpr int PER = (NF + 1023) / 1024;
    {
        u32x4 r[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j)
            r[j] = packed[min((int)threadIdx.x + 1024 * j, NF - 1)];
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if ((int)threadIdx.x + 1024 * j < NF)
                sw[threadIdx.x + 1024 * j] = r[j];
    }
    for (int i = threadIdx.x; i < 3 * NH + NOUT; i += 1024)
        sb[i] = P[i < NH ? OFF_B1 + i
                  : i < 2 * NH ? OFF_B2 + (i - NH)
                  : i < 3 * NH ? OFF_B3 + (i - 2 * NH)
                               : OFF_B4 + (i - 3 * NH)];
    __syncthreads();

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = w >> 2, f = w & 3, r = lane & 15, g = lane >> 4;
    const int64_t n_tiles = (B + 15) / 16;
    const int64_t n_sets = (n_tiles + SPLIT_TILES - 1) / SPLIT_TILES;
    const f32x4 zero{0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t set = blockIdx.x; set < n_sets; set += gridDim.x) {
        const int64_t tile = set * SPLIT_TILES + i;
        const bool tv = tile < n_tiles;
        const int64_t s = tile * 16 + r;
        // layer 1: the K x N operand is x itself (features 8g..8g+7 of sample r)
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * g + e;
            v[e] = (k < NIN && s < B) ? x[s * NIN + k] : 0.0f;
        }
        const u32x4 bx{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
        {
            const f32x4 a0 = mfma(sw[(FR_F1 + 2 * f) * 64 + lane], bx, zero);
            const f32x4 a1 = mfma(sw[(FR_F1 + 2 * f + 1) * 64 + lane], bx, zero);
            xk[0][i][f][lane] = split_epilogue<TRAIN>(a0, a1, 2 * f, 0, sb, g, cache, tile, tv, lane);
        }
        __syncthreads();
        // layers 2 and 3
#pragma unroll
        for (int layer = 1; layer <= 2; ++layer) {
            const u32x4 *fr = sw + (layer == 1 ? FR_F2 : FR_F3) * 64;
            u32x4 in[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                in[q] = xk[layer - 1][i][q][lane];
            f32x4 a0 = zero, a1 = zero;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a0 = mfma(fr[(8 * f + q) * 64 + lane], in[q], a0);
                a1 = mfma(fr[(8 * f + 4 + q) * 64 + lane], in[q], a1);
            }
            xk[layer][i][f][lane] =
                split_epilogue<TRAIN>(a0, a1, 2 * f, layer, sb, g, cache, tile, tv, lane);
            __syncthreads();
        }
        // layer 4 (rows 0..2 of the 16-row output tile), by one wave per tile
        if (f == 0) {
            f32x4 acc = zero;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc = mfma(sw[(FR_F4 + q) * 64 + lane], xk[2][i][q][lane], acc);
            if (g == 0 && s < B) {
#pragma unroll
                for (int e = 0; e < NOUT; ++e)
                    y[s * NOUT + e] = acc[e] + sb[3 * NH + e];
            }
        }
    }
}

// ---------------------------------------------------------------- backward
// v from another lane of the same 16-lane row (a DPP operand: no LDS trip)
template <int CTRL>
__device__ inline float row_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of a row, every lane receiving it: the butterfly
// over lane ^ 1, ^ 2, ^ 4, ^ 8.  After the first two steps the four lanes
// of a quad hold equal values, so the half-row mirror (lane 7 - i) stands
// for lane ^ 4, and likewise the row mirror (15 - i) for lane ^ 8.
__device__ inline float sum16(float v)
{
    v += row_lane<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += row_lane<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += row_lane<0x141>(v);  // row_half_mirror
    v += row_lane<0x140>(v);  // row_mirror
    return v;
}

__device__ inline void put(float *p, bool first, float v)
{
    *p = first ? v : *p + v;
}

__device__ inline u32x4 lds_frag(const uint16_t *base, int row, int col)
{
    return *(const u32x4 *)(base + row * BWD_ROW + col);
}

// dW tile (rows 16 tn.., cols 16 tk..) = sum over the chunk's 64 samples of
// G[n][s] H[k][s]; lane (r, g) receives rows 16 tn + 4g + e, column 16 tk + r.
__device__ inline f32x4 dw_tile(const uint16_t *G, const uint16_t *H, int tn, int tk, int lane)
{
    const int r = lane & 15, g = lane >> 4;
    f32x4 acc{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < BWD_CHUNK; kk += 32)
        acc = mfma(lds_frag(G, 16 * tn + r, kk + 8 * g), lds_frag(H, 16 * tk + r, kk + 8 * g), acc);
    return acc;
}

// Writes the bf16 transpose of a 128 x 16 register tile set (lane (r, g)
// holding v[t][e] for feature 16t + 4g + e of sample column col) into an
// LDS [feature][sample] buffer.
__device__ inline void stage_t(uint16_t *buf, const f32x4 (&v)[8], int col, int g)
{
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            buf[(16 * t + 4 * g + e) * BWD_ROW + col] = (uint16_t)bf16_bits(v[t][e]);
}

// Same, from the cached bf16 words (lane (r, g) holding the pair words of
// features 16t + 4g .. 16t + 4g + 3 of its sample).
__device__ inline void stage_tb(uint16_t *buf, const uint2 (&hw)[8], int col, int g)
{
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        uint16_t *p = buf + (16 * t + 4 * g) * BWD_ROW + col;
        p[0] = (uint16_t)(hw[t].x & 0xFFFFu);
        p[BWD_ROW] = (uint16_t)(hw[t].x >> 16);
        p[2 * BWD_ROW] = (uint16_t)(hw[t].y & 0xFFFFu);
        p[3 * BWD_ROW] = (uint16_t)(hw[t].y >> 16);
    }
}

// GELU'(z) and the bf16 activations of one hidden layer of a tile.
__device__ inline void load_cache(f32x4 (&gg)[8], uint2 (&hw)[8], const float *__restrict__ cache,
                                  int64_t tile, bool valid, int layer, int lane)
{
    float *c = const_cast<float *>(cache);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        gg[t] = valid ? *(const f32x4 *)cache_gg(c, tile, layer, t, lane)
                      : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        hw[t] = valid ? *(const uint2 *)cache_h(c, tile, layer, t, lane) : make_uint2(0u, 0u);
    }
}

// Operand of the next backward matmul from dZ tiles (same slot permutation
// as the forward pass).
__device__ inline void to_operand(u32x4 (&op)[4], const f32x4 (&d)[8])
{
#pragma unroll
    for (int q = 0; q < 4; ++q)
        op[q] = u32x4{pack2(d[2 * q][0], d[2 * q][1]), pack2(d[2 * q][2], d[2 * q][3]),
                      pack2(d[2 * q + 1][0], d[2 * q + 1][1]),
                      pack2(d[2 * q + 1][2], d[2 * q + 1][3])};
}

// Backward pass over chunks of 64 samples; each workgroup accumulates its
// chunks into its own row of `part`.  Eight waves: waves 0-3 each carry one
// 16-sample tile down the layers (dZ in registers, the transposed products
// on the matrix cores); all eight share each layer's weight-gradient tiles
// (LDS operands).  The next layer's cache entries are loaded while the
// current layer's gradient tiles run.
constexpr int BWD_THREADS = 512;
constexpr int BWD_W = BWD_THREADS / 64;

// The cached bf16 activations of one layer of a tile, into LDS rows.
__device__ inline void load_h(uint2 (&hw)[8], const float *__restrict__ cache, int64_t tile,
                              bool valid, int layer, int lane)
{
    float *c = const_cast<float *>(cache);
    const int64_t tc = valid ? tile : 0;
#pragma unroll
    for (int t = 0; t < 8; ++t)
        hw[t] = *(const uint2 *)cache_h(c, tc, layer, t, lane);
#pragma unroll
    for (int t = 0; t < 8; ++t)
        hw[t] = valid ? hw[t] : make_uint2(0u, 0u);
}

__device__ inline void load_gg(f32x4 (&gg)[8], const float *__restrict__ cache, int64_t tile,
                               bool valid, int layer, int lane)
{
    float *c = const_cast<float *>(cache);
    const int64_t tc = valid ? tile : 0;
#pragma unroll
    for (int t = 0; t < 8; ++t)
        gg[t] = *(const f32x4 *)cache_gg(c, tc, layer, t, lane);
#pragma unroll
    for (int t = 0; t < 8; ++t)
        gg[t] = valid ? gg[t] : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

// The 64 gradient tiles (16 x 16) of a 128 x 128 weight matrix, shared by
// the workgroup's waves, from the staged G (dZ^T) and H (A^T).
__device__ inline void dw_tiles_128(float *prow, int offW, bool first, const uint16_t *G,
                                    const uint16_t *H, int w, int lane)
{
    const int r = lane & 15, g = lane >> 4;
#pragma unroll 2
    for (int i = 0; i < 64 / BWD_W; ++i) {
        const int idx = w + BWD_W * i, tn = idx >> 3, tk = idx & 7;
        const f32x4 a = dw_tile(G, H, tn, tk, lane);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            put(prow + offW + (16 * tn + 4 * g + e) * NH + 16 * tk + r, first, a[e]);
    }
}

__global__ __launch_bounds__(BWD_THREADS) void k_mlp_backward(float *__restrict__ part,
                                                              const float *__restrict__ dy,
                                                              const float *__restrict__ x,
                                                              const float *__restrict__ cache,
                                                              int64_t B,
                                                              const u32x4 *__restrict__ packed,
                                                              int64_t n_chunks)
{
    __shared__ __attribute__((aligned(16))) uint16_t G[NH * BWD_ROW];
    __shared__ __attribute__((aligned(16))) uint16_t H[NH * BWD_ROW];
    __shared__ float bsum[4][NH];
    // the transposed-weight fragments (B4, B3, B2: 72 KiB) in LDS, staged
    // once with all of a thread's loads in flight
    constexpr int NBF = (FR_N - FR_B4) * 64;
    static_assert(NBF % BWD_THREADS == 0, "fragments per thread");
    __shared__ u32x4 sbw[NBF];
    {
        u32x4 rr[NBF / BWD_THREADS];
#pragma unroll
        for (int j = 0; j < NBF / BWD_THREADS; ++j)
            rr[j] = packed[FR_B4 * 64 + threadIdx.x + BWD_THREADS * j];
#pragma unroll
        for (int j = 0; j < NBF / BWD_THREADS; ++j)
            sbw[threadIdx.x + BWD_THREADS * j] = rr[j];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    const bool chain = w < 4;  // waves 0-3: one tile each
    const int col = 16 * (w & 3) + r;
    const int64_t n_tiles = (B + 15) / 16;
    float *prow = part + (int64_t)blockIdx.x * NPARAM;

    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        const bool first = chunk == blockIdx.x;
        const int64_t tile = chunk * 4 + (w & 3);
        const bool tv = tile < n_tiles;
        const int64_t s = tile * 16 + r;
        f32x4 gg[8], gn[8], dz[8];
        uint2 hw[8];
        float xin[4], d4[NOUT];
        if (chain) {
            load_gg(gg, cache, tile, tv, 2, lane);
            load_h(hw, cache, tile, tv, 2, lane);
            const int64_t sc = s < B ? s : 0;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                xin[e] = x[sc * NIN + min(4 * g + e, NIN - 1)];
#pragma unroll
            for (int e = 0; e < NOUT; ++e)
                d4[e] = dy[sc * NOUT + e];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                xin[e] = (4 * g + e < NIN && s < B) ? xin[e] : 0.0f;
#pragma unroll
            for (int e = 0; e < NOUT; ++e)
                d4[e] = s < B ? d4[e] : 0.0f;

            // ---- layer 4: dZ4 = dy
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int n = 4 * g + e;
                G[n * BWD_ROW + col] = n < NOUT ? (uint16_t)bf16_bits(d4[n < NOUT ? n : 0]) : 0;
            }
            if (g == 0) {
#pragma unroll
                for (int e = 0; e < NOUT; ++e) {
                    const float t = sum16(d4[e]);
                    if (r == 0)
                        bsum[w][e] = t;
                }
            }
            stage_tb(H, hw, col, g);
        }
        __syncthreads();
        // the next layer's cache entries, in flight during the tiles below
        if (chain) {
            load_gg(gn, cache, tile, tv, 1, lane);
            load_h(hw, cache, tile, tv, 1, lane);
        }
        // dW4 (rows 0..2 of tile 0): column tile tk = w
        {
            const int tk = w;
            const f32x4 a = dw_tile(G, H, 0, tk, lane);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (4 * g + e < NOUT)
                    put(prow + OFF_W4 + (4 * g + e) * NH + 16 * tk + r, first, a[e]);
        }
        if (threadIdx.x < NOUT)
            put(prow + OFF_B4 + threadIdx.x, first,
                ((bsum[0][threadIdx.x] + bsum[1][threadIdx.x]) + bsum[2][threadIdx.x]) +
                    bsum[3][threadIdx.x]);
        // dH3 = W4^T dZ4, dZ3 = dH3 * GELU'(z3)
        if (chain) {
            const u32x4 op4 = g == 0 ? u32x4{pack2(d4[0], d4[1]), pack2(d4[2], 0.0f), 0u, 0u}
                                     : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const f32x4 a = mfma(sbw[t * 64 + lane], op4, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    dz[t][e] = a[e] * gg[t][e];
            }
        }
        __syncthreads();

        // ---- layers 3 and 2 (weights W3, then W2)
#pragma unroll
        for (int layer = 2; layer >= 1; --layer) {
            const int offW = layer == 2 ? OFF_W3 : OFF_W2;
            const int offB = layer == 2 ? OFF_B3 : OFF_B2;
            const int frB = layer == 2 ? FR_B3 : FR_B2;
            u32x4 op[4];
            if (chain) {
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    gg[t] = gn[t];
                to_operand(op, dz);
                stage_t(G, dz, col, g);
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float v = sum16(dz[t][e]);
                        if (r == 0)
                            bsum[w][16 * t + 4 * g + e] = v;
                    }
                stage_tb(H, hw, col, g);
            }
            __syncthreads();
            if (chain && layer == 2) {  // the first layer's entries for the next round
                load_gg(gn, cache, tile, tv, 0, lane);
                load_h(hw, cache, tile, tv, 0, lane);
            }
            dw_tiles_128(prow, offW, first, G, H, w, lane);
            if (threadIdx.x < NH)
                put(prow + offB + threadIdx.x, first,
                    ((bsum[0][threadIdx.x] + bsum[1][threadIdx.x]) + bsum[2][threadIdx.x]) +
                        bsum[3][threadIdx.x]);
            // dH = W^T dZ, dZ(prev) = dH * GELU'(z(prev))
            if (chain) {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    f32x4 a{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        a = mfma(sbw[(frB - FR_B4 + t * 4 + q) * 64 + lane], op[q], a);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        dz[t][e] = a[e] * gg[t][e];
                }
            }
            __syncthreads();
        }

        // ---- layer 1: dW1 = dZ1^T x (row tile tn = w)
        if (chain) {
            stage_t(G, dz, col, g);
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float v = sum16(dz[t][e]);
                    if (r == 0)
                        bsum[w][16 * t + 4 * g + e] = v;
                }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                H[(4 * g + e) * BWD_ROW + col] = (uint16_t)bf16_bits(xin[e]);
        }
        __syncthreads();
        {
            const int tn = w;
            const f32x4 a = dw_tile(G, H, tn, 0, lane);
            if (r < NIN) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    put(prow + OFF_W1 + (16 * tn + 4 * g + e) * NIN + r, first, a[e]);
            }
        }
        if (threadIdx.x < NH)
            put(prow + OFF_B1 + threadIdx.x, first,
                ((bsum[0][threadIdx.x] + bsum[1][threadIdx.x]) + bsum[2][threadIdx.x]) +
                    bsum[3][threadIdx.x]);
        __syncthreads();
    }
}

// grad[i] = sum over the partial rows: four threads per parameter each sum
// a quarter of the rows in order, then ((q0 + q1) + q2) + q3 (a fixed
// order: deterministic).
constexpr int RED_SPLIT = 4;
__global__ __launch_bounds__(256) void k_mlp_reduce(float *__restrict__ grad,
                                                    const float *__restrict__ part, int rows)
{
    __shared__ float qs[RED_SPLIT][64];
    const int j = threadIdx.x & 63, h = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + j;
    const int per = (rows + RED_SPLIT - 1) / RED_SPLIT;
    const int w0 = h * per, w1 = min(rows, w0 + per);
    float acc = 0.0f;
    if (i < NPARAM) {
#pragma unroll 8
        for (int w = w0; w < w1; ++w)
            acc += part[(int64_t)w * NPARAM + i];
    }
    qs[h][j] = acc;
    __syncthreads();
    if (h == 0 && i < NPARAM)
        grad[i] = ((qs[0][j] + qs[1][j]) + qs[2][j]) + qs[3][j];
}

__global__ __launch_bounds__(1024) void k_mlp_mse(float *__restrict__ dy, float *__restrict__ loss,
                                                  const float *__restrict__ yv,
                                                  const float *__restrict__ tv, int64_t n)
{
    __shared__ float red[1024];
    const float scale = 2.0f / (float)n;
    float acc = 0.0f;
#pragma unroll 4
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const float d = yv[i] - tv[i];
        dy[i] = scale * d;
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int m = 512; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m)
            red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss)
        *loss = red[0] / (float)n;
}

struct AdamF {
    float lr, b1, omb1, b2, omb2, eps, c1, c2;  // omb = 1 - beta, c = 1 / (1 - beta^t)
};

// Slot p (0..31) of a K-step whose neuron is 32q + k32: the inverse of
// perm32.
__device__ inline int perm32_inv(int k32)
{
    const int k = k32 < 16 ? k32 : k32 - 16;
    return 8 * (k >> 2) + (k & 3) + (k32 < 16 ? 0 : 4);
}

// Packed bf16 element of fragment f, lane l = r + 16 (p >> 3), slot p & 7.
__device__ inline int packed_index(int f, int r, int p)
{
    return f * 512 + (r + 16 * (p >> 3)) * 8 + (p & 7);
}

// The packed elements (up to two: a forward and a transposed fragment) of
// master weight i; -1 where there is none (biases are not packed).  The
// inverse of pack_source.
__device__ inline void packed_of(int i, int &j0, int &j1)
{
    j0 = j1 = -1;
    if (i < OFF_B1) {  // W1 [128][5]: F1, K = the input feature
        const int n = i / NIN, k = i % NIN;
        j0 = packed_index(FR_F1 + (n >> 4), n & 15, k);
    } else if (i >= OFF_W2 && i < OFF_B2) {  // W2 [128][128]: F2 and B2
        const int n = (i - OFF_W2) / NH, k = (i - OFF_W2) % NH;
        j0 = packed_index(FR_F2 + (n >> 4) * 4 + (k >> 5), n & 15, perm32_inv(k & 31));
        j1 = packed_index(FR_B2 + (k >> 4) * 4 + (n >> 5), k & 15, perm32_inv(n & 31));
    } else if (i >= OFF_W3 && i < OFF_B3) {  // W3: F3 and B3
        const int n = (i - OFF_W3) / NH, k = (i - OFF_W3) % NH;
        j0 = packed_index(FR_F3 + (n >> 4) * 4 + (k >> 5), n & 15, perm32_inv(k & 31));
        j1 = packed_index(FR_B3 + (k >> 4) * 4 + (n >> 5), k & 15, perm32_inv(n & 31));
    } else if (i >= OFF_W4 && i < OFF_B4) {  // W4 [3][128]: F4 and B4
        const int o = (i - OFF_W4) / NH, k = (i - OFF_W4) % NH;
        j0 = packed_index(FR_F4 + (k >> 5), o, perm32_inv(k & 31));
        j1 = packed_index(FR_B4 + (k >> 4), k & 15, o);
    }
}

// One Adam step per master weight, whose bf16 copies in the packed
// fragments are rewritten at once (the padding keeps the zeros the first
// pack wrote).
__global__ void k_mlp_adam(float *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
                           uint16_t *__restrict__ packed, const float *__restrict__ grad, AdamF h)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM)
        return;
    const float gi = grad[i];
    const float mi = h.b1 * m[i] + h.omb1 * gi;
    const float vi = h.b2 * v[i] + h.omb2 * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float pi = P[i] - h.lr * (mi * h.c1) / (sqrtf(vi * h.c2) + h.eps);
    P[i] = pi;
    int j0, j1;
    packed_of(i, j0, j1);
    const uint16_t b = (uint16_t)bf16_bits(pi);
    if (j0 >= 0)
        packed[j0] = b;
    if (j1 >= 0)
        packed[j1] = b;
}

struct Box5 {
    float lo[5], hi[5];
};

__global__ void k_hull(uint8_t *__restrict__ fb, unsigned long long *__restrict__ counters,
                       const float *__restrict__ x, int64_t B, Box5 box)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int out = 0;
    if (b < B) {
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            const float v = x[b * NIN + i];
            if (!(v >= box.lo[i] && v <= box.hi[i]))
                out = 1;
        }
        fb[b] = (uint8_t)out;
    }
    if (counters) {
        const int c = __syncthreads_count(out);
        if (threadIdx.x == 0 && c > 0)
            atomicAdd(counters + SDM_CNT_FALLBACK, (unsigned long long)c);
    }
}

// Joint test: the per-feature box, then the cell of an occupancy grid over
// the first three features (the standardised log moments), G cells per axis
// from glo with G / (ghi - glo) cells per unit (ginv): a row whose cell no
// training input reached is out of distribution.  Single-precision steps
// in a fixed order, so the host's reading of the same rule agrees.
struct OodArgs {
    float lo[5], hi[5];
    float glo[3], ginv[3];
    int32_t G;
};

__global__ void k_ood(uint8_t *__restrict__ fb, unsigned long long *__restrict__ counters,
                      const float *__restrict__ x, int64_t B, const uint8_t *__restrict__ occ,
                      OodArgs o)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int out = 0;
    if (b < B) {
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            const float v = x[b * NIN + i];
            if (!(v >= o.lo[i] && v <= o.hi[i]))
                out = 1;
        }
        if (!out && occ) {
            int64_t cell = 0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float t = (x[b * NIN + i] - o.glo[i]) * o.ginv[i];
                int k = (int)floorf(t);
                k = k < 0 ? 0 : (k >= o.G ? o.G - 1 : k);  // the box's upper edge
                cell = cell * o.G + k;
            }
            out = occ[cell] == 0;
        }
        fb[b] = (uint8_t)out;
    }
    if (counters) {
        const int c = __syncthreads_count(out);
        if (threadIdx.x == 0 && c > 0)
            atomicAdd(counters + SDM_CNT_FALLBACK, (unsigned long long)c);
    }
}

// Fallback of the surrogate: the particles of a cell rebuilt from its
// moments.  Cell c (when selected) gets n SDs in slots [c n, c n + n) at the
// standard-normal quantiles z_i = sqrt(2) erfinv(2 (i + 1/2)/n - 1):
// v_i = e^(sigma z_i) scaled so that the mean volume is M1/M0, with sigma
// the root of R(sigma) = n sum e^(2 sigma z_i) / (sum e^(sigma z_i))^2 =
// M2 M0 / M1^2 (the sample's own second moment, matched exactly; R grows
// from 1 at sigma = 0 towards n), found by 60 bisection steps on
// [0, hi], hi the first of 1, 2, 4, .. 64 with R(hi) >= the target;
// multiplicity rint(M0 dV / n), at least 1.  Unselected cells and cells
// without positive moments get multiplicity 0 (no live SDs).  The slots'
// volumes hold the z_i while sigma is sought.
__device__ __forceinline__ double seed_ratio(const double *z, int n, double sg)
{
    double S1 = 0.0, S2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double e = exp(sg * z[i]);
        S1 += e;
        S2 += e * e;
    }
    return ((double)n * S2) / (S1 * S1);
}

__global__ void k_seed(uint64_t *__restrict__ xi, double *__restrict__ v,
                       const double *__restrict__ M, const uint8_t *__restrict__ sel,
                       int32_t n_cell, int32_t n, double dv)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cell)
        return;
    const int64_t base = c * (int64_t)n;
    double *vc = v + base;
    const double M0 = M[c * 3 + 0], M1 = M[c * 3 + 1], M2 = M[c * 3 + 2];
    if ((sel && !sel[c]) || !(M0 > 0.0 && M1 > 0.0 && M2 > 0.0)) {
        for (int i = 0; i < n; ++i) {
            xi[base + i] = 0;
            vc[i] = 0.0;
        }
        return;
    }
    const double m1 = M1 / M0;
    const double target = (M2 / M0) / (m1 * m1);
    for (int i = 0; i < n; ++i)
        vc[i] = 1.4142135623730951 * erfinv(2.0 * (((double)i + 0.5) / (double)n) - 1.0);
    double sg = 0.0;
    if (target > 1.0 && n > 1) {
        double lo = 0.0, hi = 1.0;
        while (hi < 64.0 && seed_ratio(vc, n, hi) < target)
            hi = hi * 2.0;
        for (int it = 0; it < 60; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (seed_ratio(vc, n, mid) < target)
                lo = mid;
            else
                hi = mid;
        }
        sg = 0.5 * (lo + hi);
    }
    double S = 0.0;
    for (int i = 0; i < n; ++i) {
        const double e = exp(sg * vc[i]);
        vc[i] = e;
        S += e;
    }
    const double scale = (m1 * (double)n) / S;
    const double xr = rint((M0 * dv) / (double)n);
    const uint64_t x = xr >= 1.0 ? (uint64_t)xr : 1ull;
    for (int i = 0; i < n; ++i) {
        vc[i] = vc[i] * scale;
        xi[base + i] = x;
    }
}

__global__ void k_merge(double *__restrict__ M, const double *__restrict__ src,
                        const uint8_t *__restrict__ sel, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || !sel[c])
        return;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        M[c * 3 + k] = src[c * 3 + k];
}

struct Std5 {
    double mean[5], std[5];
};

__global__ void k_features(float *__restrict__ x, const double *__restrict__ M, int64_t n,
                           double dt, double kid, Std5 st)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n)
        return;
    const double raw[5] = {log(M[c * 3 + 0]), log(M[c * 3 + 1]), log(M[c * 3 + 2]), dt, kid};
#pragma unroll
    for (int i = 0; i < 5; ++i)
        x[c * NIN + i] = (float)((raw[i] - st.mean[i]) / st.std[i]);
}

struct Std3 {
    double mean[3], std[3];
};

__global__ void k_apply(double *__restrict__ M, const float *__restrict__ yv,
                        const uint8_t *__restrict__ fb, int64_t n, double dt, Std3 st)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || (fb && fb[c]))
        return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double tend = (double)yv[c * 3 + k] * st.std[k] + st.mean[k];
        M[c * 3 + k] = M[c * 3 + k] * (1.0 + dt * tend);
    }
}

inline int grid_for(int64_t n, int per)
{
    return (int)((n + per - 1) / per);
}

int check_mlp(const sdm_ctx *ctx, const sdm_mlp *w)
{
    if (!ctx || !w || !w->params || !w->packed)
        return fail(SDM_E_INVALID, "null context or network");
    if (((uintptr_t)w->packed & 15) != 0)
        return fail(SDM_E_INVALID, "packed weights must be 16-byte aligned");
    return SDM_OK;
}

}  // namespace

extern "C" {

int sdm_mlp_pack(sdm_ctx *ctx, const sdm_mlp *w, hipStream_t stream)
{
    if (int rc = check_mlp(ctx, w))
        return rc;
    SDM_TRY
    hipLaunchKernelGGL(k_mlp_pack, dim3(grid_for(FR_N * 256, 256)), dim3(256), 0, stream,
                       (uint32_t *)w->packed, (const float *)w->params);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_mlp_forward(sdm_ctx *ctx, float *y, float *cache, const float *x, int64_t B,
                    const sdm_mlp *w, hipStream_t stream)
{
    if (int rc = check_mlp(ctx, w))
        return rc;
    REQUIRE(B >= 0, "B < 0");
    if (B == 0)
        return SDM_OK;
    REQUIRE(y && x, "null y or x");
    REQUIRE(B <= ((int64_t)1 << 34), "B too large");
    SDM_TRY
    const int64_t tiles = (B + 15) / 16;
    if (tiles <= SPLIT_MAX_TILES) {
        // up to a few tiles per SIMD: four waves per tile
        const int64_t sets = (tiles + SPLIT_TILES - 1) / SPLIT_TILES;
        const dim3 grid(sets < 256 ? (unsigned)sets : 256u);
        if (cache)
            hipLaunchKernelGGL(k_mlp_forward_split<true>, grid, dim3(1024), 0, stream, y, cache,
                               x, B, (const u32x4 *)w->packed, w->params);
        else
            hipLaunchKernelGGL(k_mlp_forward_split<false>, grid, dim3(1024), 0, stream, y, cache,
                               x, B, (const u32x4 *)w->packed, w->params);
    } else {
        // one wave per tile; inference takes two tiles at a time (larger
        // batches only), training one, writing its training cache
        const int S = cache ? 1 : 2;
        const int64_t want = (tiles + 4 * S - 1) / (4 * S);
        const int grid = (int)(want < FWD_GRID_MAX ? want : FWD_GRID_MAX);
        if (cache)
            hipLaunchKernelGGL((k_mlp_forward<1, true>), dim3(grid), dim3(256), 0, stream, y,
                               cache, x, B, (const u32x4 *)w->packed, w->params);
        else
            hipLaunchKernelGGL((k_mlp_forward<2, false>), dim3(grid), dim3(256), 0, stream, y,
                               cache, x, B, (const u32x4 *)w->packed, w->params);
    }
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_mlp_backward(sdm_ctx *ctx, float *grad, const float *dy, const float *x,
                     const float *cache, int64_t B, const sdm_mlp *w, hipStream_t stream)
{
    if (int rc = check_mlp(ctx, w))
        return rc;
    REQUIRE(grad, "grad is NULL");
    REQUIRE(B >= 0, "B < 0");
    REQUIRE(B == 0 || (dy && x && cache), "null dy, x or cache");
    REQUIRE(B <= ((int64_t)1 << 34), "B too large");
    SDM_TRY
    const int64_t chunks = (B + BWD_CHUNK - 1) / BWD_CHUNK;
    const int rows = (int)(chunks < PART_ROWS_MAX ? chunks : PART_ROWS_MAX);
    if (rows > ctx->mlp_part_rows) {
        SDM_HIP(hipDeviceSynchronize());
        if (ctx->mlp_part)
            SDM_HIP(hipFree(ctx->mlp_part));
        ctx->mlp_part = nullptr;
        ctx->mlp_part_rows = 0;
        SDM_HIP(hipMalloc(&ctx->mlp_part, (size_t)rows * NPARAM * sizeof(float)));
        ctx->mlp_part_rows = rows;
    }
    if (rows > 0)
        hipLaunchKernelGGL(k_mlp_backward, dim3(rows), dim3(BWD_THREADS), 0, stream,
                           ctx->mlp_part, dy, x, cache, B, (const u32x4 *)w->packed, chunks);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(NPARAM, 64)), dim3(64 * RED_SPLIT), 0, stream,
                       grad, ctx->mlp_part, rows);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_mlp_mse(sdm_ctx *ctx, float *dy, float *loss, const float *y, const float *t, int64_t B,
                hipStream_t stream)
{
    REQUIRE(ctx, "ctx is NULL");
    REQUIRE(B > 0, "B must be positive");
    REQUIRE(dy && y && t, "null dy, y or t");
    SDM_TRY
    hipLaunchKernelGGL(k_mlp_mse, dim3(1), dim3(1024), 0, stream, dy, loss, y, t, B * NOUT);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_mlp_adam(sdm_ctx *ctx, const sdm_mlp *w, const sdm_mlp_opt *opt, const float *grad,
                 const sdm_adam_hp *hp, hipStream_t stream)
{
    if (int rc = check_mlp(ctx, w))
        return rc;
    REQUIRE(opt && opt->m && opt->v && grad && hp, "null optimiser state, grad or hp");
    REQUIRE(hp->t >= 1, "Adam step t must be >= 1");
    REQUIRE(hp->beta1 >= 0 && hp->beta1 < 1 && hp->beta2 >= 0 && hp->beta2 < 1,
            "betas out of [0, 1)");
    SDM_TRY
    AdamF h;
    h.lr = (float)hp->lr;
    h.b1 = (float)hp->beta1;
    h.omb1 = (float)(1.0 - hp->beta1);
    h.b2 = (float)hp->beta2;
    h.omb2 = (float)(1.0 - hp->beta2);
    h.eps = (float)hp->eps;
    h.c1 = (float)(1.0 / (1.0 - pow(hp->beta1, (double)hp->t)));
    h.c2 = (float)(1.0 / (1.0 - pow(hp->beta2, (double)hp->t)));
    hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(NPARAM, 256)), dim3(256), 0, stream, w->params,
                       opt->m, opt->v, (uint16_t *)w->packed, grad, h);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_hull_check(sdm_ctx *ctx, uint8_t *fallback, uint64_t *counters_dev, const float *x,
                   int64_t B, const float *lo, const float *hi, hipStream_t stream)
{
    REQUIRE(ctx && lo && hi, "null ctx, lo or hi");
    REQUIRE(B >= 0, "B < 0");
    if (B == 0)
        return SDM_OK;
    REQUIRE(fallback && x, "null fallback or x");
    SDM_TRY
    Box5 box;
    for (int i = 0; i < NIN; ++i) {
        box.lo[i] = lo[i];
        box.hi[i] = hi[i];
    }
    hipLaunchKernelGGL(k_hull, dim3(grid_for(B, 256)), dim3(256), 0, stream, fallback,
                       (unsigned long long *)counters_dev, x, B, box);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_mlp_features(sdm_ctx *ctx, float *x, const double *M, int64_t n, double dt,
                     int32_t kernel_id, const float *mean, const float *std, hipStream_t stream)
{
    REQUIRE(ctx && mean && std, "null ctx, mean or std");
    REQUIRE(n >= 0, "n < 0");
    if (n == 0)
        return SDM_OK;
    REQUIRE(x && M, "null x or M");
    SDM_TRY
    Std5 st;
    for (int i = 0; i < NIN; ++i) {
        st.mean[i] = mean[i];
        st.std[i] = std[i];
    }
    hipLaunchKernelGGL(k_features, dim3(grid_for(n, 256)), dim3(256), 0, stream, x, M, n, dt,
                       (double)kernel_id, st);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_mlp_apply(sdm_ctx *ctx, double *M, const float *y, const uint8_t *fallback, int64_t n,
                  double dt, const float *mean, const float *std, hipStream_t stream)
{
    REQUIRE(ctx && mean && std, "null ctx, mean or std");
    REQUIRE(n >= 0, "n < 0");
    if (n == 0)
        return SDM_OK;
    REQUIRE(M && y, "null M or y");
    SDM_TRY
    Std3 st;
    for (int i = 0; i < 3; ++i) {
        st.mean[i] = mean[i];
        st.std[i] = std[i];
    }
    hipLaunchKernelGGL(k_apply, dim3(grid_for(n, 256)), dim3(256), 0, stream, M, y, fallback, n,
                       dt, st);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_ood_check(sdm_ctx *ctx, uint8_t *fallback, uint64_t *counters_dev, const float *x,
                  int64_t B, const float *lo, const float *hi, const uint8_t *occ, int32_t G,
                  const float *glo, const float *ginv, hipStream_t stream)
{
    REQUIRE(ctx && lo && hi, "null ctx, lo or hi");
    REQUIRE(B >= 0, "B < 0");
    REQUIRE(!occ || (G >= 1 && G <= 256 && glo && ginv), "occupancy grid: G in [1, 256] "
            "with glo and ginv");
    if (B == 0)
        return SDM_OK;
    REQUIRE(fallback && x, "null fallback or x");
    SDM_TRY
    OodArgs o{};
    for (int i = 0; i < NIN; ++i) {
        o.lo[i] = lo[i];
        o.hi[i] = hi[i];
    }
    if (occ) {
        for (int i = 0; i < 3; ++i) {
            o.glo[i] = glo[i];
            o.ginv[i] = ginv[i];
        }
        o.G = G;
    }
    hipLaunchKernelGGL(k_ood, dim3(grid_for(B, 256)), dim3(256), 0, stream, fallback,
                       (unsigned long long *)counters_dev, x, B, occ, o);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_seed_from_moments(sdm_ctx *ctx, uint64_t *xi, double *v, const double *M,
                          const uint8_t *select, int32_t n_cell, int32_t n_per_cell, double dv,
                          hipStream_t stream)
{
    REQUIRE(ctx, "null ctx");
    REQUIRE(n_cell >= 0 && n_per_cell >= 1 && n_per_cell <= 1 << 20, "sizes out of range");
    REQUIRE(dv > 0 && std::isfinite(dv), "dv must be positive");
    if (n_cell == 0)
        return SDM_OK;
    REQUIRE(xi && v && M, "null xi, v or M");
    SDM_TRY
    hipLaunchKernelGGL(k_seed, dim3(grid_for(n_cell, 64)), dim3(64), 0, stream, xi, v, M,
                       select, n_cell, n_per_cell, dv);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

int sdm_moments_merge(sdm_ctx *ctx, double *M, const double *M_src, const uint8_t *select,
                      int64_t n, hipStream_t stream)
{
    REQUIRE(ctx, "null ctx");
    REQUIRE(n >= 0, "n < 0");
    if (n == 0)
        return SDM_OK;
    REQUIRE(M && M_src && select, "null M, M_src or select");
    SDM_TRY
    hipLaunchKernelGGL(k_merge, dim3(grid_for(n, 256)), dim3(256), 0, stream, M, M_src, select,
                       n);
    SDM_HIP(hipGetLastError());
    SDM_CATCH
}

}  // extern "C"
