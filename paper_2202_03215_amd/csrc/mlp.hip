// mlp.hip -- gfx950 kernels of the learned closure network (5-64-64-64-2,
// tanh), BF16 operands with FP32 accumulation on the matrix cores.
//
// Section IV of the paper closes the fluid equations (3)-(4) with the
// drift-diffusion fluxes (12)-(13); here a small network predicts the
// electron flux and energy flux from local moments instead.  The kernels:
//   k_mlp_pack     FP32 master parameters -> BF16 operand layouts + FP32 biases
//   k_mlp_fwd      inference over n samples (optionally keeping activations)
//   k_mlp_fwdbwd   training pass 1: forward, loss, back-propagated gradients
//                  of every layer's pre-activations (stored for pass 2)
//   k_mlp_wgrad    training pass 2: per-block partial weight/bias gradients
//                  (activation^T x gradient, reduced over samples on MFMA)
//   k_mlp_reduce   fixed-order sum of the partials (deterministic gradient)
//   k_mlp_adam     Adam update of the FP32 master parameters, then re-pack
//
// Matrix-core tile: v_mfma_f32_16x16x32_bf16, D(16x16) += A(16x32) B(32x16).
// Lane l holds A[l%16][8(l/16) .. 8(l/16)+7], B[8(l/16) .. +7][l%16] and
// D[4(l/16) .. 4(l/16)+3][l%16].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/pc_mlp.h"

namespace pcmlp {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 5, kH = 64, kOut = 2;
constexpr int kBlock = 256;   // 4 waves
constexpr int kTile = 16;     // samples per wave tile
constexpr int kChunk = 32;    // samples per weight-gradient step (MFMA K)

// offsets of the flat FP32 parameter vector (row-major W[in][out])
constexpr int oW1 = 0, oB1 = oW1 + kIn * kH, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH * kH, oW4 = oB3 + kH, oB4 = oW4 + kH * kOut, kParams = oB4 + kOut;
static_assert(kParams == PC_MLP_PARAMS, "parameter count");

// operand layouts: forward B operands are W^T rows (8 consecutive inputs of
// one output unit); backward B operands are W rows (8 consecutive outputs of
// one input unit); K and N are padded with zeros.
struct alignas(16) PackedFwd {
    bf16 w1t[kH][32];   // [out][in, padded 5 -> 32]
    bf16 w2t[kH][kH];
    bf16 w3t[kH][kH];
    bf16 w4t[16][kH];   // [out, padded 2 -> 16][in]
    float b1[kH], b2[kH], b3[kH], b4[16];
};
struct Packed : PackedFwd {
    bf16 w2[kH][kH];    // [in][out]
    bf16 w3[kH][kH];
    bf16 w4[kH][32];    // [in][out, padded 2 -> 32]
};

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ int lane() { return __lane_id(); }

// copy (the forward part of) the packed parameters into LDS (whole block)
template <class T>
__device__ __forceinline__ void stage_params(T& s, const Packed* __restrict__ g)
{
    static_assert(sizeof(T) % 16 == 0, "16-byte copies");
    const int4* src = reinterpret_cast<const int4*>(static_cast<const T*>(g));
    int4* dst = reinterpret_cast<int4*>(&s);
    for (int k = threadIdx.x; k < int(sizeof(T) / 16); k += blockDim.x) dst[k] = src[k];
}

// One dense layer for a 16-sample tile held row-major in LDS (act[16][K]):
// out[s][u] = sum_k act[s][k] W[k][u] + b[u] for the 4 N-tiles of 64 units,
// computed transposed (out^T = W^T act^T: the weights are the A operand, the
// activations the B operand), so that lane l holds units nt 16 + 4(l/16) ..
// + 3 of sample l % 16: four consecutive units of one row.
template <int K>
__device__ __forceinline__ void layer64(const bf16 (*act)[K], const bf16 (*wt)[K], const float* b, f32x4 acc[4])
{
    const int l = lane();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = *reinterpret_cast<const f32x4*>(&b[nt * 16 + 4 * (l >> 4)]);
#pragma unroll
    for (int kt = 0; kt < K / 32; ++kt) {
        const bf16x8 xb = ld8(&act[l & 15][kt * 32 + 8 * (l >> 4)]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma(ld8(&wt[nt * 16 + (l & 15)][kt * 32 + 8 * (l >> 4)]), xb, acc[nt]);
    }
}

// tanh for BF16 activations: 1 - 2 / (1 + e^(2x)), e^(2x) as 2^(2x log2 e) on
// the hardware exp2, the quotient on its reciprocal, the last step one fused
// multiply-add (exact at both ends: e^(2x) overflows to infinity for large x,
// giving 1; underflows to 0 for very negative x, giving -1).  With exp2 and
// the reciprocal each within one ulp, and r = 1/(1 + e) in (0, 1], the error
// is at most 2 r (2^-23 + 2^-24 + 2^-23) + 2^-24 |tanh x| <= 6.6e-7 absolute
// (3.6e-7 near zero, where r is 1/2); the subsequent BF16 rounding (2^-9
// relative) dominates except within that distance of a rounding point.
__device__ __forceinline__ float tanh_bf(float x)
{
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);   // 2 log2(e) x
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
}

// tanh of the accumulators (layer64's layout), rounded to BF16, into a
// row-major LDS tile (and optionally to global memory, row-major
// [sample][64]): four consecutive units per lane, one 8-byte store each
__device__ __forceinline__ void tanh_store(const f32x4 acc[4], bf16 (*act)[kH], bf16* __restrict__ g, int64_t s0,
                                           int64_t n)
{
    const int l = lane();
    const int r = l & 15;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int u = nt * 16 + 4 * (l >> 4);
        bf16x4 h;
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = bf16(tanh_bf(acc[nt][i]));
        *reinterpret_cast<bf16x4*>(&act[r][u]) = h;
        if (g != nullptr && s0 + r < n) *reinterpret_cast<bf16x4*>(&g[(s0 + r) * kH + u]) = h;
    }
}

// input tile: 16 samples x 5 features -> BF16, padded to 32
__device__ __forceinline__ void load_x(const float* __restrict__ x, int64_t s0, int64_t n, bf16 (*xs)[32])
{
    const int l = lane();
    for (int k = l; k < kTile * 32; k += 64) {
        const int r = k >> 5, c = k & 31;
        float v = 0.0f;
        if (c < kIn && s0 + r < n) v = x[(s0 + r) * kIn + c];
        xs[r][c] = bf16(v);
    }
}

struct alignas(16) WaveLds {
    bf16 x[kTile][32];
    bf16 h1[kTile][kH];
    bf16 h2[kTile][kH];
    bf16 h3[kTile][kH];
    bf16 dz[kTile][kH];   // back-propagated gradient of the current layer
};

// forward of one tile; leaves the activations in w
// (activations are stored to g1..g3 for samples below nstore: n for the
// caller's hidden output, the padded count for the training stores)
__device__ __forceinline__ void forward_tile(const PackedFwd& P, WaveLds& w, const float* __restrict__ x, int64_t s0,
                                             int64_t n, int64_t nstore, bf16* __restrict__ g1,
                                             bf16* __restrict__ g2, bf16* __restrict__ g3, f32x4 out[1])
{
    f32x4 acc[4];
    load_x(x, s0, n, w.x);
    // each wave owns its LDS tile: the fences order one lane's writes before
    // other lanes' reads of the same wave (LDS operations complete in order)
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    layer64<32>(w.x, P.w1t, P.b1, acc);
    tanh_store(acc, w.h1, g1, s0, nstore);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    layer64<kH>(w.h1, P.w2t, P.b2, acc);
    tanh_store(acc, w.h2, g2, s0, nstore);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    layer64<kH>(w.h2, P.w3t, P.b3, acc);
    tanh_store(acc, w.h3, g3, s0, nstore);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    // output layer: one N-tile (units 0, 1 real)
    const int l = lane();
    const float bias = P.b4[l & 15];
    f32x4 o = f32x4{bias, bias, bias, bias};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
        o = mfma(ld8(&w.h3[l & 15][kt * 32 + 8 * (l >> 4)]), ld8(&P.w4t[l & 15][kt * 32 + 8 * (l >> 4)]), o);
    out[0] = o;
}

// Inference layout.  LDS rows of the weights and of the activation tile are
// padded by 16 bytes: a 16x32 operand fragment is read by lanes l % 16 = row
// at one column offset, and an unpadded row pitch of 64 or 128 bytes puts all
// sixteen rows on the same banks; with a pitch of 80 or 144 bytes each group
// of eight lanes covers all banks once.  Each wave keeps one activation tile:
// a layer reads its inputs into registers before any of its outputs exist,
// and the LDS operations of one wave complete in issue order.
constexpr int kFwdBlock = 512;   // 8 waves
constexpr int kPad = 8;          // bf16 elements of row padding
constexpr int kK1 = 32 + kPad, kK2 = kH + kPad;
struct alignas(16) FwdParams {
    bf16 w1t[kH][kK1];
    bf16 w2t[kH][kK2];
    bf16 w3t[kH][kK2];
    bf16 w4t[16][kK2];
    float b1[kH], b2[kH], b3[kH], b4[16];
};

__device__ __forceinline__ void stage_fwd(FwdParams& s, const PackedFwd* __restrict__ g)
{
    for (int k = threadIdx.x; k < kH * 4; k += blockDim.x) {
        const int r = k >> 2, c = (k & 3) * 8;
        *reinterpret_cast<bf16x8*>(&s.w1t[r][c]) = ld8(&g->w1t[r][c]);
    }
    for (int k = threadIdx.x; k < kH * 8; k += blockDim.x) {
        const int r = k >> 3, c = (k & 7) * 8;
        *reinterpret_cast<bf16x8*>(&s.w2t[r][c]) = ld8(&g->w2t[r][c]);
        *reinterpret_cast<bf16x8*>(&s.w3t[r][c]) = ld8(&g->w3t[r][c]);
    }
    for (int k = threadIdx.x; k < 16 * 8; k += blockDim.x) {
        const int r = k >> 3, c = (k & 7) * 8;
        *reinterpret_cast<bf16x8*>(&s.w4t[r][c]) = ld8(&g->w4t[r][c]);
    }
    for (int k = threadIdx.x; k < kH; k += blockDim.x) {
        s.b1[k] = g->b1[k];
        s.b2[k] = g->b2[k];
        s.b3[k] = g->b3[k];
    }
    if (threadIdx.x < 16) s.b4[threadIdx.x] = g->b4[threadIdx.x];
}

// The first layer's B operand is x^T: lane l < 16 holds the five features of
// sample l of the tile (K padded to 32 with zeros), the other lanes zeros, so
// the inputs go from global memory straight into registers.  The loads are
// unconditional (index clamped into the array, value zeroed outside it), so
// that the next tile's loads stay in flight while this tile is computed.
__device__ __forceinline__ void fetch_x(const float* __restrict__ x, int64_t s0, int64_t n, float v[kIn])
{
    const int l = lane();
    const int64_t e = (s0 + (l & 15)) * kIn, end = n * kIn;
#pragma unroll
    for (int c = 0; c < kIn; ++c) {
        const int64_t i = e + c;
        const float a = x[i < end ? i : end - 1];
        v[c] = (l < 16 && i < end) ? a : 0.0f;
    }
}

// compiler-only ordering of the wave's LDS accesses (no wait instruction)
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// tanh of a layer's accumulators into the wave's tile (row = sample, four
// consecutive units per lane and N-tile), optionally also to global memory
__device__ __forceinline__ void act_store(const f32x4 acc[4], bf16 (*a)[kK2], bf16* __restrict__ g, int64_t s0,
                                          int64_t n)
{
    const int l = lane(), r = l & 15;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int u = nt * 16 + 4 * (l >> 4);
        bf16x4 h;
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = bf16(tanh_bf(acc[nt][i]));
        *reinterpret_cast<bf16x4*>(&a[r][u]) = h;
        if (g != nullptr && s0 + r < n) *reinterpret_cast<bf16x4*>(&g[(s0 + r) * kH + u]) = h;
    }
}

// one hidden layer (64 -> 64) from the wave's tile, transposed as in layer64
__device__ __forceinline__ void hidden_layer(const bf16 (*a)[kK2], const bf16 (*wt)[kK2], const float* b, f32x4 acc[4])
{
    const int l = lane(), r = l & 15, c = 8 * (l >> 4);
    const bf16x8 x0 = ld8(&a[r][c]), x1 = ld8(&a[r][32 + c]);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 v = *reinterpret_cast<const f32x4*>(&b[nt * 16 + 4 * (l >> 4)]);
        v = mfma(ld8(&wt[nt * 16 + r][c]), x0, v);
        acc[nt] = mfma(ld8(&wt[nt * 16 + r][32 + c]), x1, v);
    }
}

__global__ __launch_bounds__(kBlock) void k_mlp_pack(const float* __restrict__ m, Packed* __restrict__ p)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bf16 z = bf16(0.0f);
    if (t < kH * 32) {   // w1t[out][in], w4[in][out]
        const int o = t / 32, i = t % 32;
        p->w1t[o][i] = i < kIn ? bf16(m[oW1 + i * kH + o]) : z;
        const int ii = t / 32, oo = t % 32;
        p->w4[ii][oo] = oo < kOut ? bf16(m[oW4 + ii * kOut + oo]) : z;
    }
    if (t < kH * kH) {
        const int o = t / kH, i = t % kH;
        p->w2t[o][i] = bf16(m[oW2 + i * kH + o]);
        p->w3t[o][i] = bf16(m[oW3 + i * kH + o]);
        p->w2[o][i] = bf16(m[oW2 + o * kH + i]);   // row o = input unit
        p->w3[o][i] = bf16(m[oW3 + o * kH + i]);
    }
    if (t < 16 * kH) {
        const int o = t / kH, i = t % kH;
        p->w4t[o][i] = o < kOut ? bf16(m[oW4 + i * kOut + o]) : z;
    }
    if (t < kH) {
        p->b1[t] = m[oB1 + t];
        p->b2[t] = m[oB2 + t];
        p->b3[t] = m[oB3 + t];
    }
    if (t < 16) p->b4[t] = t < kOut ? m[oB4 + t] : 0.0f;
}

// inference: y[n][2]; hidden (optional) = three [n][64] BF16 activation arrays
__global__ __launch_bounds__(kFwdBlock) void k_mlp_fwd(const Packed* __restrict__ gp, const float* __restrict__ x,
                                                       int64_t n, float* __restrict__ y, bf16* __restrict__ hidden)
{
    __shared__ FwdParams P;
    __shared__ bf16 tile[kFwdBlock / 64][kTile][kK2];
    stage_fwd(P, gp);
    __syncthreads();
    bf16 (*a)[kK2] = tile[threadIdx.x >> 6];
    const int l = lane(), r = l & 15, c = 8 * (l >> 4);
    const int64_t tiles = (n + kTile - 1) / kTile;
    const int64_t t0 = int64_t(blockIdx.x) * (kFwdBlock / 64) + (threadIdx.x >> 6);
    const int64_t stride = int64_t(gridDim.x) * (kFwdBlock / 64);
    bf16* const h2 = hidden ? hidden + n * kH : nullptr;
    bf16* const h3 = hidden ? hidden + 2 * n * kH : nullptr;
    float xv[kIn];
    fetch_x(x, t0 * kTile, n, xv);
    for (int64_t t = t0; t < tiles; t += stride) {
        const int64_t s0 = t * kTile;
        bf16x8 xb;
#pragma unroll
        for (int k = 0; k < kIn; ++k) xb[k] = bf16(xv[k]);
#pragma unroll
        for (int k = kIn; k < 8; ++k) xb[k] = bf16(0.0f);
        fetch_x(x, s0 + stride * kTile, n, xv);   // the next tile's inputs, in flight meanwhile
        f32x4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            acc[nt] = mfma(ld8(&P.w1t[nt * 16 + r][c]), xb,
                           *reinterpret_cast<const f32x4*>(&P.b1[nt * 16 + 4 * (l >> 4)]));
        act_store(acc, a, hidden, s0, n);
        lds_order();
        hidden_layer(a, P.w2t, P.b2, acc);
        lds_order();
        act_store(acc, a, h2, s0, n);
        lds_order();
        hidden_layer(a, P.w3t, P.b3, acc);
        lds_order();
        act_store(acc, a, h3, s0, n);
        lds_order();
        // output layer, not transposed: lane l holds samples 4(l/16) .. + 3 of unit l % 16
        const float bias = P.b4[r];
        f32x4 o = f32x4{bias, bias, bias, bias};
        o = mfma(ld8(&a[r][c]), ld8(&P.w4t[r][c]), o);
        o = mfma(ld8(&a[r][32 + c]), ld8(&P.w4t[r][32 + c]), o);
        if (r < kOut)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t s = s0 + 4 * (l >> 4) + i;
                if (s < n) y[s * kOut + r] = o[i];
            }
        lds_order();
    }
}

// Training pass 1 over tiles: forward, squared error, gradients of the
// pre-activations dz4 = bf16(2 (y - t) / (2 n)), dz_l = bf16(dz_{l+1} W^T (1 - h^2)).
// Stores (row-major, samples padded to a multiple of 32 with zeros):
// xs [np][16] (BF16 inputs, padded), h1..h3 [np][64], dz1..dz3 [np][64],
// dz4 [np][16]; per-block partial sums of the squared error.
struct TrainStores {
    bf16 *xs, *h1, *h2, *h3, *dz1, *dz2, *dz3, *dz4;
    float* loss_part;
};

__global__ __launch_bounds__(kBlock) void k_mlp_fwdbwd(const Packed* __restrict__ gp, const float* __restrict__ x,
                                                       const float* __restrict__ tg, int64_t n, int64_t np,
                                                       TrainStores S)
{
    __shared__ Packed P;
    __shared__ WaveLds wl[kBlock / 64];
    __shared__ float red[kBlock / 64];
    stage_params(P, gp);
    __syncthreads();
    WaveLds& w = wl[threadIdx.x >> 6];
    const int l = lane();
    const float scale = 2.0f / float(double(n) * kOut);
    float sq = 0.0f;
    const int64_t tiles = np / kTile;
    for (int64_t t = int64_t(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6); t < tiles;
         t += int64_t(gridDim.x) * (kBlock / 64)) {
        const int64_t s0 = t * kTile;
        f32x4 o[1];
        forward_tile(P, w, x, s0, n, np, S.h1, S.h2, S.h3, o);
        // inputs as BF16 (16 columns) for the weight gradient of layer 1
        for (int k = l; k < kTile * 16; k += 64) {
            const int r = k >> 4, c = k & 15;
            S.xs[(s0 + r) * 16 + c] = w.x[r][c];
        }
        // padded samples (n <= s < np) have zero inputs and zero gradients dz,
        // so they add nothing to any weight or bias gradient
        // dz4 and the squared error (units 0, 1)
        bf16 (*dz4)[kH] = w.dz;   // first 32 columns used: [16][32]
        {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 4 * (l >> 4) + i, u = l & 15;
                const int64_t s = s0 + r;
                float d = 0.0f;
                if (u < kOut && s < n) {
                    const float e = o[0][i] - tg[s * kOut + u];
                    sq += e * e;
                    d = scale * e;
                }
                const bf16 db = bf16(d);
                dz4[r][u] = db;
                dz4[r][u + 16] = bf16(0.0f);
                S.dz4[s * 16 + u] = db;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        // dz3 = bf16((dz4 W4^T) (1 - h3^2)), K = 32 (2 real outputs)
        f32x4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            acc[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            acc[nt] = mfma(ld8(&dz4[l & 15][8 * (l >> 4)]), ld8(&P.w4[nt * 16 + (l & 15)][8 * (l >> 4)]), acc[nt]);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        const bf16(*hs[3])[kH] = {w.h1, w.h2, w.h3};
        bf16* gdz[3] = {S.dz1, S.dz2, S.dz3};
        for (int layer = 2; layer >= 0; --layer) {
            // acc holds d loss / d activation of hidden layer `layer` (0-based)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 4 * (l >> 4) + i, u = nt * 16 + (l & 15);
                    const float h = float(hs[layer][r][u]);
                    const bf16 d = (s0 + r < n) ? bf16(acc[nt][i] * (1.0f - h * h)) : bf16(0.0f);
                    w.dz[r][u] = d;
                    gdz[layer][(s0 + r) * kH + u] = d;
                }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            if (layer == 0) break;
            const bf16(*wb)[kH] = layer == 2 ? P.w3 : P.w2;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
                const bf16x8 a = ld8(&w.dz[l & 15][kt * 32 + 8 * (l >> 4)]);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[nt] = mfma(a, ld8(&wb[nt * 16 + (l & 15)][kt * 32 + 8 * (l >> 4)]), acc[nt]);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        }
    }
    // block sum of the squared error (fixed order: lanes, then waves)
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off);
    if (l == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) S.loss_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Training pass 2: block b sums activation^T x gradient over its sample range
// (chunks of 32 samples staged transposed in LDS) into partial[b][0..8833].
struct ChunkLds {
    bf16 x[16][kChunk];     // [feature][sample]
    bf16 h[3][kH][kChunk];
    bf16 dz[3][kH][kChunk];
    bf16 dz4[16][kChunk];
};

__device__ __forceinline__ void stage_t(bf16 (*dst)[kChunk], const bf16* __restrict__ src, int64_t s0, int width)
{
    // src row-major [sample][width] -> dst [feature][sample], 32 samples
    for (int k = threadIdx.x; k < kChunk * width; k += blockDim.x) {
        const int s = k / width, f = k % width;
        dst[f][s] = src[(s0 + s) * width + f];
    }
}

__global__ __launch_bounds__(kBlock) void k_mlp_wgrad(TrainStores S, int64_t np, float* __restrict__ partial)
{
    __shared__ ChunkLds c;
    const int wv = threadIdx.x >> 6, l = lane();
    const int64_t chunks = np / kChunk;
    const int64_t per = (chunks + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = int64_t(blockIdx.x) * per;
    const int64_t c1 = c0 + per < chunks ? c0 + per : chunks;
    // 40 output tiles: layer 1 (1 x 4), layer 2 (4 x 4), layer 3 (4 x 4), layer 4 (4 x 1);
    // wave wv owns tiles wv, wv + 4, ...
    f32x4 acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;   // bias gradient of parameter slot threadIdx.x (0..193)
    for (int64_t ch = c0; ch < c1; ++ch) {
        const int64_t s0 = ch * kChunk;
        __syncthreads();
        stage_t(c.x, S.xs, s0, 16);
        stage_t(c.h[0], S.h1, s0, kH);
        stage_t(c.h[1], S.h2, s0, kH);
        stage_t(c.h[2], S.h3, s0, kH);
        stage_t(c.dz[0], S.dz1, s0, kH);
        stage_t(c.dz[1], S.dz2, s0, kH);
        stage_t(c.dz[2], S.dz3, s0, kH);
        stage_t(c.dz4, S.dz4, s0, 16);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const int tile = wv + 4 * k;
            const bf16 (*A)[kChunk];
            const bf16 (*B)[kChunk];
            int mt, nt;
            if (tile < 4) { A = c.x; B = c.dz[0]; mt = 0; nt = tile; }
            else if (tile < 20) { A = c.h[0]; B = c.dz[1]; mt = (tile - 4) >> 2; nt = (tile - 4) & 3; }
            else if (tile < 36) { A = c.h[1]; B = c.dz[2]; mt = (tile - 20) >> 2; nt = (tile - 20) & 3; }
            else { A = c.h[2]; B = c.dz4; mt = tile - 36; nt = 0; }
            acc[k] = mfma(ld8(&A[mt * 16 + (l & 15)][8 * (l >> 4)]), ld8(&B[nt * 16 + (l & 15)][8 * (l >> 4)]),
                          acc[k]);
        }
        // bias gradients: column sums of dz over the chunk
        const int t = threadIdx.x;
        if (t < 3 * kH + kOut) {
            const bf16* col = t < 3 * kH ? &c.dz[t / kH][t % kH][0] : &c.dz4[t - 3 * kH][0];
            float s = 0.0f;
            for (int q = 0; q < kChunk; ++q) s += float(col[q]);
            bsum += s;
        }
    }
    float* out = partial + int64_t(blockIdx.x) * kParams;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const int tile = wv + 4 * k;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * (l >> 4) + i, nn = l & 15;   // D[m][nn] of the tile
            if (tile < 4) {
                const int in = m, o = tile * 16 + nn;
                if (in < kIn) out[oW1 + in * kH + o] = acc[k][i];
            } else if (tile < 36) {
                const int q = tile < 20 ? tile - 4 : tile - 20;
                const int in = (q >> 2) * 16 + m, o = (q & 3) * 16 + nn;
                out[(tile < 20 ? oW2 : oW3) + in * kH + o] = acc[k][i];
            } else {
                const int in = (tile - 36) * 16 + m, o = nn;
                if (o < kOut) out[oW4 + in * kOut + o] = acc[k][i];
            }
        }
    }
    const int t = threadIdx.x;
    if (t < 3 * kH) out[(t < kH ? oB1 : t < 2 * kH ? oB2 : oB3) + t % kH] = bsum;
    else if (t < 3 * kH + kOut) out[oB4 + t - 3 * kH] = bsum;
}

// grad[p] = sum over blocks b (in order) of partial[b][p]; loss likewise
__global__ __launch_bounds__(kBlock) void k_mlp_reduce(const float* __restrict__ partial, int nb,
                                                       const float* __restrict__ loss_part, int nl,
                                                       int64_t n, float* __restrict__ grad, float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kParams) {
        float s = 0.0f;
        for (int b = 0; b < nb; ++b) s += partial[int64_t(b) * kParams + p];
        grad[p] = s;
    }
    if (p == 0 && loss != nullptr) {
        float s = 0.0f;
        for (int b = 0; b < nl; ++b) s += loss_part[b];
        *loss = s / float(double(n) * kOut);
    }
}

// omb1 = 1 - beta1, omb2 = 1 - beta2 and the bias corrections c1, c2 come
// from the host in double precision, rounded once
__global__ __launch_bounds__(kBlock) void k_mlp_adam(float* __restrict__ m, float* __restrict__ mom,
                                                     float* __restrict__ vel, const float* __restrict__ g,
                                                     float lr, float b1, float b2, float omb1, float omb2, float eps,
                                                     float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const float gp = g[p];
    const float mm = b1 * mom[p] + omb1 * gp;
    const float vv = b2 * vel[p] + omb2 * (gp * gp);
    mom[p] = mm;
    vel[p] = vv;
    m[p] = m[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace pcmlp

// ---------------------------------------------------------------- C ABI
using namespace pcmlp;

namespace {
thread_local const char* g_mlp_err = "";
constexpr int64_t pad32(int64_t n) { return (n + kChunk - 1) / kChunk * kChunk; }
int grid_for(int64_t tiles) { return int(tiles < 2048 ? (tiles < 1 ? 1 : tiles) : 2048); }
constexpr int kWgradBlocks = 256;

struct ScratchLayout {
    int64_t xs, h1, h2, h3, dz1, dz2, dz3, dz4, loss, partial, total;
};
constexpr ScratchLayout scratch_layout(int64_t n)
{
    const int64_t np = pad32(n);
    ScratchLayout L{};
    int64_t o = 0;
    auto take = [&](int64_t bytes) constexpr {
        const int64_t at = o;
        o = (o + bytes + 255) & ~int64_t(255);
        return at;
    };
    L.xs = take(np * 16 * 2);
    L.h1 = take(np * kH * 2);
    L.h2 = take(np * kH * 2);
    L.h3 = take(np * kH * 2);
    L.dz1 = take(np * kH * 2);
    L.dz2 = take(np * kH * 2);
    L.dz3 = take(np * kH * 2);
    L.dz4 = take(np * 16 * 2);
    L.loss = take(2048 * 4);
    L.partial = take(int64_t(kWgradBlocks) * kParams * 4);
    L.total = o;
    return L;
}
constexpr int64_t kNoAllocBytes = scratch_layout(PC_MLP_NOALLOC_MAX_BATCH).total;
}  // namespace

// Training scratch of the allocation-free gradient (pc_mlp_grad_noalloc):
// one copy per device, placed by the code object loader and held until the
// process ends.  In host code `scratch` is only a handle for
// hipGetSymbolAddress; kernels receive the device address it returns.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
pc_status noalloc_scratch(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        g_mlp_err = "no current device (or device index above 63)";
        return PC_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_mlp_err = "hipGetSymbolAddress of the training scratch failed";
            return PC_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PC_OK;
}

// the gradient pass of pc_mlp_grad with its scratch at b (layout L)
pc_status grad_into(const void* packed, const float* x, const float* target, int64_t n, float* grad, float* loss,
                    char* b, const ScratchLayout& L, hipStream_t st)
{
    TrainStores S;
    S.xs = reinterpret_cast<bf16*>(b + L.xs);
    S.h1 = reinterpret_cast<bf16*>(b + L.h1);
    S.h2 = reinterpret_cast<bf16*>(b + L.h2);
    S.h3 = reinterpret_cast<bf16*>(b + L.h3);
    S.dz1 = reinterpret_cast<bf16*>(b + L.dz1);
    S.dz2 = reinterpret_cast<bf16*>(b + L.dz2);
    S.dz3 = reinterpret_cast<bf16*>(b + L.dz3);
    S.dz4 = reinterpret_cast<bf16*>(b + L.dz4);
    S.loss_part = reinterpret_cast<float*>(b + L.loss);
    float* partial = reinterpret_cast<float*>(b + L.partial);
    const int64_t np = pad32(n);
    const int g1 = grid_for((np / kTile + 3) / 4);
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3(g1), dim3(kBlock), 0, st, static_cast<const Packed*>(packed), x, target,
                       n, np, S);
    const int64_t chunks = np / kChunk;
    const int g2 = int(chunks < kWgradBlocks ? chunks : kWgradBlocks);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(g2), dim3(kBlock), 0, st, S, np, partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + kBlock - 1) / kBlock), dim3(kBlock), 0, st, partial, g2,
                       S.loss_part, g1, n, grad, loss);
    return hipGetLastError() == hipSuccess ? PC_OK : PC_ERR_HIP;
}
}  // namespace

extern "C" {

pc_status pc_mlp_query(int64_t max_batch, pc_mlp_sizes* out)
{
    if (!out || max_batch < 1 || max_batch > (int64_t(1) << 31)) {
        g_mlp_err = "bad batch size";
        return PC_ERR_INVALID_ARG;
    }
    out->params = kParams;
    out->packed_bytes = int64_t(sizeof(Packed));
    out->scratch_bytes = scratch_layout(max_batch).total;
    return PC_OK;
}

pc_status pc_mlp_pack(const float* master, void* packed, void* stream)
{
    if (!master || !packed) {
        g_mlp_err = "null argument";
        return PC_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_mlp_pack, dim3((kH * kH + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), master, static_cast<Packed*>(packed));
    return hipGetLastError() == hipSuccess ? PC_OK : PC_ERR_HIP;
}

pc_status pc_mlp_forward(const void* packed, const float* x, int64_t n, float* y, uint16_t* hidden, void* stream)
{
    if (!packed || n < 0 || (n > 0 && (!x || !y)) || n > (int64_t(1) << 31)) {
        g_mlp_err = "bad forward arguments";
        return PC_ERR_INVALID_ARG;
    }
    if (n == 0) return PC_OK;
    const int64_t tiles = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(grid_for((tiles + 7) / 8)), dim3(kFwdBlock), 0,
                       static_cast<hipStream_t>(stream), static_cast<const Packed*>(packed), x, n, y,
                       reinterpret_cast<bf16*>(hidden));
    return hipGetLastError() == hipSuccess ? PC_OK : PC_ERR_HIP;
}

pc_status pc_mlp_grad(const void* packed, const float* x, const float* target, int64_t n, float* grad, float* loss,
                      void* scratch, size_t scratch_bytes, void* stream)
{
    if (!packed || !x || !target || !grad || !scratch || n < 1 || n > (int64_t(1) << 31)) {
        g_mlp_err = "bad gradient arguments";
        return PC_ERR_INVALID_ARG;
    }
    const ScratchLayout L = scratch_layout(n);
    if (int64_t(scratch_bytes) < L.total) {
        g_mlp_err = "scratch too small";
        return PC_ERR_WORKSPACE;
    }
    return grad_into(packed, x, target, n, grad, loss, static_cast<char*>(scratch), L,
                     static_cast<hipStream_t>(stream));
}

pc_status pc_mlp_grad_noalloc(const void* packed, const float* x, const float* target, int64_t n, float* grad,
                              float* loss, void* stream)
{
    if (!packed || !x || !target || !grad || n < 1) {
        g_mlp_err = "bad gradient arguments";
        return PC_ERR_INVALID_ARG;
    }
    if (n > PC_MLP_NOALLOC_MAX_BATCH) {
        g_mlp_err = "batch above PC_MLP_NOALLOC_MAX_BATCH (16384 samples) for the allocation-free gradient";
        return PC_ERR_INVALID_ARG;
    }
    void* base = nullptr;
    const pc_status s = noalloc_scratch(&base);
    if (s != PC_OK) return s;
    return grad_into(packed, x, target, n, grad, loss, static_cast<char*>(base), scratch_layout(n),
                     static_cast<hipStream_t>(stream));
}

pc_status pc_mlp_adam(float* master, float* m, float* v, const float* grad, int64_t step, double lr, double beta1,
                      double beta2, double eps, void* packed, void* stream)
{
    if (!master || !m || !v || !grad || step < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
        !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0)) {
        g_mlp_err = "bad Adam arguments";
        return PC_ERR_INVALID_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float c1 = float(1.0 - std::pow(beta1, double(step)));
    const float c2 = float(1.0 - std::pow(beta2, double(step)));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + kBlock - 1) / kBlock), dim3(kBlock), 0, st, master, m, v, grad,
                       float(lr), float(beta1), float(beta2), float(1.0 - beta1), float(1.0 - beta2), float(eps), c1,
                       c2);
    if (packed)
        hipLaunchKernelGGL(k_mlp_pack, dim3((kH * kH + kBlock - 1) / kBlock), dim3(kBlock), 0, st, master,
                           static_cast<Packed*>(packed));
    return hipGetLastError() == hipSuccess ? PC_OK : PC_ERR_HIP;
}

const char* pc_mlp_last_error(void) { return g_mlp_err; }

}  // extern "C"
