// Per-particle MLP that gives the solver its initial guess: forward,
// backward and Adam on gfx950's BF16 matrix cores (v_mfma_f32_16x16x32_bf16)
// with FP32 accumulation.  Not part of the paper, which names better initial
// guesses as future work (Sections "Conclusions and future work" and
// "Implementation notes").
//
// Network (one sample = one fluid particle and one velocity component):
//   x[4] -> 64 -> 64 -> 64 -> o[3], ReLU on the hidden layers,
//   pred = o0 B0 + o1 B1 + o2 B2 with basis B = (b_c, u_c, (u - A u)_c) / U.
// The two 64x64 layers, their data gradients and their weight gradients run
// on MFMA, 16 samples per tile; the 4->64 and 64->3 layers run on the vector
// ALU in FP32 in training and on MFMA with two-part BF16 inputs in inference.
// Weights enter every product as BF16; the inputs of the 64x64 products
// (activations and gradient signals) are rounded to BF16 as well.
//
// MFMA fragment layout (lane l, g = l / 16, c = l % 16, r = 0..3): the
// output D[4g + r][c]; the operands of one 16x16x32 step carry 8 values of K
// per lane, A[c][k] and B[k][c] for the lane group's 8 slots.  The kernels
// assign slot i of group g to K index 16 (i / 4) + 4 g + i % 4 of the step:
// two 16-wide halves, each in the layout of a D output (rows 4g + r), so a
// product's output (or two tiles' worth of samples) becomes the next
// product's operand by concatenating two 4-value fragments, with no
// shuffle.  A and B use the same assignment, so the product is exact in it.
#include <algorithm>
#include <cmath>

#include "mlp.hpp"
#include "operator_kernels.hpp"

namespace sph {
namespace mlp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// The operand of one 16x16x32 step from two 4-value fragments (K slots
// 0..3 and 4..7 of the lane group).
__device__ inline bf16x8 cat8(bf16x4 lo, bf16x4 hi) {
    return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}
__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int kWaves = 4;             // waves per block
constexpr int kThreads = kWaves * kWave;
constexpr int kPad = 65;              // padded row of the per-wave transpose tile

// Orders a wave's own LDS writes before its later LDS reads by other lanes
// (every tile and output staging area belongs to one wave, so waves of a
// block never wait for each other after the parameters are loaded).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint16_t f2bf(float f) {  // nearest, ties to even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline float rbf(float f) { return bf2f(f2bf(f)); }

struct Smem {
    uint16_t w2[kH * kH], w2t[kH * kH], w3[kH * kH], w3t[kH * kH];  // [in][out] and [out][in]
    float w1[kIn * kH];     // BF16-rounded values
    float w4[kH * kOut];    // BF16-rounded values
    float b1[kH], b2[kH], b3[kH], b4[4];
    float tile[kWaves][16 * kPad];  // per-wave transpose / activation tile
    float go[kWaves][16 * 4];       // per-wave outputs o or output gradients
};

__device__ inline void load_params(Smem& sm, const float* __restrict__ p) {
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) {
        const int in = i / kH, out = i % kH;
        const uint16_t v2 = f2bf(p[kOW2 + i]), v3 = f2bf(p[kOW3 + i]);
        sm.w2[i] = v2;
        sm.w2t[out * kH + in] = v2;
        sm.w3[i] = v3;
        sm.w3t[out * kH + in] = v3;
    }
    for (int i = threadIdx.x; i < kIn * kH; i += blockDim.x) sm.w1[i] = rbf(p[kOW1 + i]);
    for (int i = threadIdx.x; i < kH * kOut; i += blockDim.x) sm.w4[i] = rbf(p[kOW4 + i]);
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        sm.b1[i] = p[kOB1 + i];
        sm.b2[i] = p[kOB2 + i];
        sm.b3[i] = p[kOB3 + i];
    }
    if (threadIdx.x < kOut) sm.b4[threadIdx.x] = p[kOB4 + threadIdx.x];
    __syncthreads();
}

// B fragment of a forward product h W (B[k][n] = W[k][n]), k-step s, n-tile t.
__device__ inline bf16x4 bfrag_fwd(const uint16_t* __restrict__ wt, int s, int t, int g, int c) {
    const uint16_t* q = wt + (16 * t + c) * kH + 16 * s + 4 * g;
    bf16x4 v;
    v[0] = (short)q[0];
    v[1] = (short)q[1];
    v[2] = (short)q[2];
    v[3] = (short)q[3];
    return v;
}
// B fragment of a data-gradient product dz W^T (B[k][n] = W[n][k]).
__device__ inline bf16x4 bfrag_bwd(const uint16_t* __restrict__ w, int s, int t, int g, int c) {
    const uint16_t* q = w + (16 * t + c) * kH + 16 * s + 4 * g;
    bf16x4 v;
    v[0] = (short)q[0];
    v[1] = (short)q[1];
    v[2] = (short)q[2];
    v[3] = (short)q[3];
    return v;
}

// D-layout values v[t][r] (row 4g + r, column 16t + c) -> A fragments
// (row c, columns 16s + 4g + r) through the wave's LDS tile, BF16-rounded.
__device__ inline void d_to_a(float* tile, const float (&v)[4][4], bf16x4 (&a)[4], int g, int c) {
    for (int t = 0; t < 4; ++t)
        for (int r = 0; r < 4; ++r) tile[(4 * g + r) * kPad + 16 * t + c] = v[t][r];
    wave_sync();
    for (int s = 0; s < 4; ++s)
        for (int r = 0; r < 4; ++r) a[s][r] = (short)f2bf(tile[c * kPad + 16 * s + 4 * g + r]);
    wave_sync();
}

// One 64x64 product on MFMA: out[t] (D layout) = A (16x64) x Wfrag, two
// 32-wide K steps (16-wide blocks 2s and 2s + 1).
template <bool FWD>
__device__ inline void mm64(const bf16x4 (&a)[4], const uint16_t* __restrict__ w, int g, int c, f32x4 (&acc)[4]) {
    for (int t = 0; t < 4; ++t) {
        acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int s = 0; s < 2; ++s) {
            const bf16x4 b0 = FWD ? bfrag_fwd(w, 2 * s, t, g, c) : bfrag_bwd(w, 2 * s, t, g, c);
            const bf16x4 b1 = FWD ? bfrag_fwd(w, 2 * s + 1, t, g, c) : bfrag_bwd(w, 2 * s + 1, t, g, c);
            acc[t] = mfma32(cat8(a[2 * s], a[2 * s + 1]), cat8(b0, b1), acc[t]);
        }
    }
}

// First layer for one sample x: z1 at column col.
__device__ inline float layer1(const Smem& sm, const float (&x)[4], int col) {
    float z = sm.b1[col];
    for (int f = 0; f < kIn; ++f) z = __builtin_fmaf(x[f], sm.w1[f * kH + col], z);
    return z;
}

// State of one 16-sample tile kept for the backward pass.
struct Tile {
    float xA[4];        // features of sample row c
    float xD[4][4];     // features of sample rows 4g + r
    float bD[4][3];     // basis of rows 4g + r (for the output gradient)
    float tD[4];        // targets of rows 4g + r
    float h1[4][4];     // D layout (post-ReLU)
    float h2[4][4];
    float h3[4][4];
};

// Forward pass of one tile; leaves h3 in the wave's LDS tile and the
// outputs o in sm.go[wave].  Returns nothing; the caller reads sm.go.
__device__ inline void tile_forward(Smem& sm, Tile& T, int wave, int g, int c) {
    float* tile = sm.tile[wave];
    // layer 1 in A layout (input of the first MFMA product) and in D layout
    bf16x4 a[4];
    for (int s = 0; s < 4; ++s)
        for (int r = 0; r < 4; ++r) a[s][r] = (short)f2bf(fmaxf(layer1(sm, T.xA, 16 * s + 4 * g + r), 0.f));
    for (int t = 0; t < 4; ++t)
        for (int r = 0; r < 4; ++r) T.h1[t][r] = fmaxf(layer1(sm, T.xD[r], 16 * t + c), 0.f);
    f32x4 acc[4];
    mm64<true>(a, sm.w2t, g, c, acc);
    for (int t = 0; t < 4; ++t)
        for (int r = 0; r < 4; ++r) T.h2[t][r] = fmaxf(acc[t][r] + sm.b2[16 * t + c], 0.f);
    d_to_a(tile, T.h2, a, g, c);
    mm64<true>(a, sm.w3t, g, c, acc);
    for (int t = 0; t < 4; ++t)
        for (int r = 0; r < 4; ++r) T.h3[t][r] = fmaxf(acc[t][r] + sm.b3[16 * t + c], 0.f);
    // layer 4 on the vector ALU: h3 through the LDS tile
    for (int t = 0; t < 4; ++t)
        for (int r = 0; r < 4; ++r) tile[(4 * g + r) * kPad + 16 * t + c] = T.h3[t][r];
    wave_sync();
    const int lane = threadIdx.x % kWave;
    if (lane < 16 * kOut) {
        const int row = lane / kOut, k = lane % kOut;
        float o = sm.b4[k];
        for (int col = 0; col < kH; ++col) o = __builtin_fmaf(tile[row * kPad + col], sm.w4[col * kOut + k], o);
        sm.go[wave][row * 4 + k] = o;
    }
    wave_sync();
}

// Loads sample `s` (or zeros when s < 0) into the lane's tile rows.
__device__ inline void load_tile(Tile& T, const float* __restrict__ S, const int32_t* __restrict__ idx,
                                 int64_t base, int64_t count, int g, int c) {
    auto sample = [&](int64_t k) -> const float* {
        if (k >= count) return nullptr;
        const int64_t s = idx ? (int64_t)idx[base + k] : base + k;
        return S + s * kSample;
    };
    const float* pa = sample(c);
    for (int f = 0; f < 4; ++f) T.xA[f] = pa ? pa[f] : 0.f;
    for (int r = 0; r < 4; ++r) {
        const float* pd = sample(4 * g + r);
        for (int f = 0; f < 4; ++f) T.xD[r][f] = pd ? pd[f] : 0.f;
        for (int k = 0; k < 3; ++k) T.bD[r][k] = pd ? pd[4 + k] : 0.f;
        T.tD[r] = pd ? pd[7] : 0.f;
    }
}

// Inference: out[s] = (o0, o1, o2, pred) for samples [0, n).  All four
// products run on MFMA, transposed, Z^T = W^T H^T, with the 16 samples of a
// tile on the MFMA N dimension: a product's output then sits in registers
// exactly as the next product's B operand (lane (g, c) holds features
// 16t + 4g + r of sample c), so no LDS transpose is needed; the weights of
// the 64x64 layers, as A operands, stay in registers for the whole launch,
// those of the first and last layers in LDS.  The 64x64 layers take BF16
// weights and BF16 layer inputs, as in the training kernel.  The first and
// last layers take their inputs as sums of BF16 parts against the same BF16
// weight: the features as three parts, which hold an FP32 value exactly (K
// slots 4g + r, g = 0, 1, 2, carry part g of feature r), so layer 1 equals
// the training kernel's FP32 layer up to the order of its FP32 sums (its
// output is rounded to BF16 next, where a less accurate input would flip
// roundings); the last hidden layer as two parts, to 2^-16 relative (one K
// step per part; the output is not rounded again).  The training kernel
// evaluates these two layers in FP32 on the vector ALU.
// Two floats to packed BF16, nearest-even (the hardware conversion of
// gfx950; the same rounding as f2bf on finite values).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 hbf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t pk_bf16(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, hbf16x2));
}
__device__ inline bf16x4 bf16x4_of(float v0, float v1, float v2, float v3) {
    return __builtin_bit_cast(bf16x4, u32x2{pk_bf16(v0, v1), pk_bf16(v2, v3)});
}
// The four values' BF16 parts: hi = nearest BF16, lo = BF16 of v - hi (the
// remainder v - hi is exact in FP32); rem receives v - hi - lo, exact too.
__device__ inline void bf16x4_split(const float (&v)[4], bf16x4& hi, bf16x4& lo, float (&rem)[4]) {
    hi = bf16x4_of(v[0], v[1], v[2], v[3]);
    for (int r = 0; r < 4; ++r) rem[r] = v[r] - bf2f((uint16_t)hi[r]);
    lo = bf16x4_of(rem[0], rem[1], rem[2], rem[3]);
    for (int r = 0; r < 4; ++r) rem[r] -= bf2f((uint16_t)lo[r]);
}

struct alignas(16) InferSmem {
    alignas(16) float b1[kH];
    alignas(16) float b2[kH];
    alignas(16) float b3[kH];
    alignas(16) float b4[4];
    alignas(16) bf16x8 a1[4][kWave];  // A operands of layer 1 (tile t, lane)
    alignas(16) bf16x8 a4[2][kWave];  // A operands of layer 4 (K step s, lane)
};

// At most 128 registers, so that four waves share a SIMD (the operands' set-up
// spills a few values once per block, none in the tile loop).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_mlp_infer(const float* __restrict__ S, int64_t n,
                                                        const float* __restrict__ p, float* __restrict__ out) {
    __shared__ __align__(16) InferSmem sm;
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        sm.b1[i] = p[kOB1 + i];
        sm.b2[i] = p[kOB2 + i];
        sm.b3[i] = p[kOB3 + i];
    }
    if (threadIdx.x < 4) sm.b4[threadIdx.x] = threadIdx.x < kOut ? p[kOB4 + threadIdx.x] : 0.f;
    // A operands: step s of output tile t holds W[in][16t + c] (W stored
    // [in][out]) for the lane group's K slots, in = 32s + 16 (i / 4) + 4g + i % 4
    const int lane = threadIdx.x % kWave, g = lane / 16, c = lane % 16;
    bf16x8 a2[4][2], a3[4][2];
    for (int t = 0; t < 4; ++t)
        for (int s = 0; s < 2; ++s) {
            bf16x4 lo2, hi2, lo3, hi3;
            for (int r = 0; r < 4; ++r) {
                const int in = 32 * s + 4 * g + r, o = 16 * t + c;
                lo2[r] = (short)f2bf(p[kOW2 + in * kH + o]);
                hi2[r] = (short)f2bf(p[kOW2 + (in + 16) * kH + o]);
                lo3[r] = (short)f2bf(p[kOW3 + in * kH + o]);
                hi3[r] = (short)f2bf(p[kOW3 + (in + 16) * kH + o]);
            }
            a2[t][s] = cat8(lo2, hi2);
            a3[t][s] = cat8(lo3, hi3);
        }
    // layer 1: K slot 4g + r (g = 0, 1, 2: the three parts) is feature r;
    // the other slots are zero.  Layer 4: output row c (< 3) of
    // W4^T, K = the 64 hidden units.  Both kept in LDS (one copy per lane
    // index, shared by the block's waves), read once per tile.
    const bf16x4 z4 = {0, 0, 0, 0};
    if (threadIdx.x < kWave) {
        for (int t = 0; t < 4; ++t) {
            bf16x4 w = z4;
            if (g < 3)
                for (int r = 0; r < 4; ++r) w[r] = (short)f2bf(p[kOW1 + r * kH + 16 * t + c]);
            sm.a1[t][lane] = cat8(w, z4);
        }
        for (int s = 0; s < 2; ++s) {
            bf16x4 lo4 = z4, hi4 = z4;
            if (c < kOut)
                for (int r = 0; r < 4; ++r) {
                    const int in = 32 * s + 4 * g + r;
                    lo4[r] = (short)f2bf(p[kOW4 + in * kOut + c]);
                    hi4[r] = (short)f2bf(p[kOW4 + (in + 16) * kOut + c]);
                }
            sm.a4[s][lane] = cat8(lo4, hi4);
        }
    }
    __syncthreads();
    const int64_t ntiles = ceil_div(n, (int64_t)16);
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave; tile < ntiles; tile += nw) {
        // re-read the small LDS tables every tile rather than keeping them
        // in registers (which would leave room for fewer waves per SIMD)
        __asm__ volatile("" ::: "memory");
        const int64_t smp = tile * 16 + c;
        const bool valid = smp < n;
        const float4 x = valid ? *reinterpret_cast<const float4*>(S + smp * kSample) : float4{0.f, 0.f, 0.f, 0.f};
        // layer 1 on MFMA, bias, ReLU, BF16: the B operand of layer 2
        bf16x4 xh, xm;
        float xr[4];
        bf16x4_split({x.x, x.y, x.z, x.w}, xh, xm, xr);
        const bf16x4 xl = bf16x4_of(xr[0], xr[1], xr[2], xr[3]);  // exact: at most 8 bits remain
        const bf16x8 b1 = cat8(g == 0 ? xh : (g == 1 ? xm : (g == 2 ? xl : z4)), z4);
        bf16x4 h[4];
        for (int t = 0; t < 4; ++t) {
            const f32x4 z = mfma32(sm.a1[t][lane], b1, f32x4{0.f, 0.f, 0.f, 0.f});
            const float4 b = *reinterpret_cast<const float4*>(&sm.b1[16 * t + 4 * g]);
            h[t] = bf16x4_of(fmaxf(z[0] + b.x, 0.f), fmaxf(z[1] + b.y, 0.f), fmaxf(z[2] + b.z, 0.f),
                             fmaxf(z[3] + b.w, 0.f));
        }
        // layer 2 on MFMA, bias, ReLU, BF16: the B operand of layer 3
        f32x4 acc[4];
        for (int t = 0; t < 4; ++t) {
            acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int s = 0; s < 2; ++s) acc[t] = mfma32(a2[t][s], cat8(h[2 * s], h[2 * s + 1]), acc[t]);
        }
        for (int t = 0; t < 4; ++t) {
            const float4 b = *reinterpret_cast<const float4*>(&sm.b2[16 * t + 4 * g]);
            const float bb[4] = {b.x, b.y, b.z, b.w};
            h[t] = bf16x4_of(fmaxf(acc[t][0] + bb[0], 0.f), fmaxf(acc[t][1] + bb[1], 0.f),
                             fmaxf(acc[t][2] + bb[2], 0.f), fmaxf(acc[t][3] + bb[3], 0.f));
        }
        // layer 3 on MFMA, bias, ReLU, split into BF16 parts: the B operands
        // of layer 4
        for (int t = 0; t < 4; ++t) {
            acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int s = 0; s < 2; ++s) acc[t] = mfma32(a3[t][s], cat8(h[2 * s], h[2 * s + 1]), acc[t]);
        }
        bf16x4 hh[4], hl[4];
        for (int t = 0; t < 4; ++t) {
            const float4 b = *reinterpret_cast<const float4*>(&sm.b3[16 * t + 4 * g]);
            const float v[4] = {fmaxf(acc[t][0] + b.x, 0.f), fmaxf(acc[t][1] + b.y, 0.f),
                                fmaxf(acc[t][2] + b.z, 0.f), fmaxf(acc[t][3] + b.w, 0.f)};
            float rem[4];
            bf16x4_split(v, hh[t], hl[t], rem);
        }
        // layer 4 on MFMA: rows 0-2 of the output tile (lanes of group 0)
        f32x4 o4 = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int s = 0; s < 2; ++s) {
            const bf16x8 w4 = sm.a4[s][lane];
            o4 = mfma32(w4, cat8(hh[2 * s], hh[2 * s + 1]), o4);
            o4 = mfma32(w4, cat8(hl[2 * s], hl[2 * s + 1]), o4);
        }
        if (g == 0 && valid) {
            const float o0 = o4[0] + sm.b4[0], o1 = o4[1] + sm.b4[1], o2 = o4[2] + sm.b4[2];
            const float4 bs = *reinterpret_cast<const float4*>(S + smp * kSample + 4);
            float pred = o0 * bs.x;
            pred = __builtin_fmaf(o1, bs.y, pred);
            pred = __builtin_fmaf(o2, bs.z, pred);
            *reinterpret_cast<float4*>(out + smp * 4) = float4{o0, o1, o2, pred};
        }
    }
}

// Forward and backward of a batch (sample ids idx[0, batch)); every wave
// writes its partial gradient (kNParam values) and its partial sum of
// squared errors to part[global wave][0 .. kNParam].
__global__ __launch_bounds__(kThreads) void k_mlp_train(const float* __restrict__ S,
                                                        const int32_t* __restrict__ idx, int64_t batch,
                                                        const float* __restrict__ params,
                                                        float* __restrict__ part, int32_t tiles_per_wave) {
    __shared__ Smem sm;
    load_params(sm, params);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, g = lane / 16, c = lane % 16;
    const int64_t gw = (int64_t)blockIdx.x * kWaves + wave;
    const float inv_m = 2.0f / (float)batch;
    float* tile = sm.tile[wave];
    f32x4 gW2[4][4], gW3[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) gW2[i][j] = gW3[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float gW1[4][4] = {}, gb1[4] = {}, gb2[4] = {}, gb3[4] = {};
    float gW4[3] = {0.f, 0.f, 0.f}, gb4 = 0.f, sse = 0.f;
    // The weight gradients h^T dz sum over the samples (K); one 32-wide
    // step takes two tiles, so the operands of every even tile wait for the
    // next tile (or for zeros after the last one).
    bf16x4 pah3[4], pbz3[4], pah2[4], pbz2[4];
    bool pend = false;
    const auto wgrad = [&](f32x4 (&gW)[4][4], bf16x4 (&pa)[4], bf16x4 (&pb)[4], const bf16x4 (&ah)[4],
                           const bf16x4 (&bz)[4]) {
        if (!pend) {
            for (int t = 0; t < 4; ++t) {
                pa[t] = ah[t];
                pb[t] = bz[t];
            }
            return;
        }
        for (int mt = 0; mt < 4; ++mt)
            for (int nt = 0; nt < 4; ++nt) gW[mt][nt] = mfma32(cat8(pa[mt], ah[mt]), cat8(pb[nt], bz[nt]), gW[mt][nt]);
    };
    for (int q = 0; q < tiles_per_wave; ++q) {
        const int64_t base = (gw * tiles_per_wave + q) * 16;
        Tile T;
        load_tile(T, S, idx, base, batch - base, g, c);
        tile_forward(sm, T, wave, g, c);
        // output gradient g_o = (2/m) (pred - t) B of rows 0..15 (lanes 0..15
        // read their own o and overwrite it)
        if (lane < 16) {
            const int64_t k = base + lane;
            float go[3] = {0.f, 0.f, 0.f};
            if (k < batch) {
                const float* ps = S + (int64_t)idx[k] * kSample;
                const float* o = &sm.go[wave][lane * 4];
                float pred = o[0] * ps[4];
                pred = __builtin_fmaf(o[1], ps[5], pred);
                pred = __builtin_fmaf(o[2], ps[6], pred);
                const float err = pred - ps[7];
                sse = __builtin_fmaf(err, err, sse);
                for (int j = 0; j < 3; ++j) go[j] = inv_m * err * ps[4 + j];
            }
            for (int j = 0; j < 3; ++j) sm.go[wave][lane * 4 + j] = go[j];
        }
        wave_sync();
        const float* GO = sm.go[wave];
        // layer 4: dW4[col][k] += sum_row h3[row][col] g_o[row][k] (h3 still in the tile)
        for (int row = 0; row < 16; ++row) {
            const float h = tile[row * kPad + lane];
            for (int k = 0; k < 3; ++k) gW4[k] = __builtin_fmaf(h, GO[row * 4 + k], gW4[k]);
        }
        if (lane < 3)
            for (int row = 0; row < 16; ++row) gb4 += GO[row * 4 + lane];
        // dz3 (D layout)
        float dz[4][4];
        for (int t = 0; t < 4; ++t)
            for (int r = 0; r < 4; ++r) {
                const int row = 4 * g + r, col = 16 * t + c;
                float d = GO[row * 4 + 0] * sm.w4[col * kOut + 0];
                d = __builtin_fmaf(GO[row * 4 + 1], sm.w4[col * kOut + 1], d);
                d = __builtin_fmaf(GO[row * 4 + 2], sm.w4[col * kOut + 2], d);
                dz[t][r] = T.h3[t][r] > 0.f ? d : 0.f;
            }
        wave_sync();
        // layer 3: weight gradient h2^T dz3, bias gradient, data gradient dz3 W3^T
        for (int t = 0; t < 4; ++t)
            for (int r = 0; r < 4; ++r) gb3[t] += dz[t][r];
        {
            bf16x4 ah[4], bz[4];
            for (int t = 0; t < 4; ++t)
                for (int r = 0; r < 4; ++r) {
                    ah[t][r] = (short)f2bf(T.h2[t][r]);
                    bz[t][r] = (short)f2bf(dz[t][r]);
                }
            wgrad(gW3, pah3, pbz3, ah, bz);
        }
        bf16x4 a[4];
        d_to_a(tile, dz, a, g, c);
        f32x4 acc[4];
        mm64<false>(a, sm.w3, g, c, acc);
        for (int t = 0; t < 4; ++t)
            for (int r = 0; r < 4; ++r) dz[t][r] = T.h2[t][r] > 0.f ? acc[t][r] : 0.f;
        // layer 2
        for (int t = 0; t < 4; ++t)
            for (int r = 0; r < 4; ++r) gb2[t] += dz[t][r];
        {
            bf16x4 ah[4], bz[4];
            for (int t = 0; t < 4; ++t)
                for (int r = 0; r < 4; ++r) {
                    ah[t][r] = (short)f2bf(T.h1[t][r]);
                    bz[t][r] = (short)f2bf(dz[t][r]);
                }
            wgrad(gW2, pah2, pbz2, ah, bz);
        }
        d_to_a(tile, dz, a, g, c);
        mm64<false>(a, sm.w2, g, c, acc);
        // layer 1
        for (int t = 0; t < 4; ++t)
            for (int r = 0; r < 4; ++r) {
                const float d = T.h1[t][r] > 0.f ? acc[t][r] : 0.f;
                gb1[t] += d;
                for (int f = 0; f < 4; ++f) gW1[f][t] = __builtin_fmaf(T.xD[r][f], d, gW1[f][t]);
            }
        pend = !pend;
    }
    if (pend) {
        // the last tile's weight gradients with a zero partner
        const bf16x4 z4{0, 0, 0, 0};
        const bf16x4 zero[4] = {z4, z4, z4, z4};
        wgrad(gW3, pah3, pbz3, zero, zero);
        wgrad(gW2, pah2, pbz2, zero, zero);
    }
    // write this wave's partial gradient
    float* P = part + gw * (int64_t)(kNParam + 1);
    for (int mt = 0; mt < 4; ++mt)
        for (int nt = 0; nt < 4; ++nt)
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * mt + 4 * g + r, col = 16 * nt + c;
                P[kOW2 + row * kH + col] = gW2[mt][nt][r];
                P[kOW3 + row * kH + col] = gW3[mt][nt][r];
            }
    for (int t = 0; t < 4; ++t) {
        float v1 = gb1[t], v2 = gb2[t], v3 = gb3[t];
        float w[4] = {gW1[0][t], gW1[1][t], gW1[2][t], gW1[3][t]};
        for (int off = 16; off < kWave; off <<= 1) {
            v1 += __shfl_xor(v1, off, kWave);
            v2 += __shfl_xor(v2, off, kWave);
            v3 += __shfl_xor(v3, off, kWave);
            for (int f = 0; f < 4; ++f) w[f] += __shfl_xor(w[f], off, kWave);
        }
        if (g == 0) {
            P[kOB1 + 16 * t + c] = v1;
            P[kOB2 + 16 * t + c] = v2;
            P[kOB3 + 16 * t + c] = v3;
            for (int f = 0; f < 4; ++f) P[kOW1 + f * kH + 16 * t + c] = w[f];
        }
    }
    for (int k = 0; k < 3; ++k) P[kOW4 + lane * kOut + k] = gW4[k];
    if (lane < 3) P[kOB4 + lane] = gb4;
    for (int off = 1; off < 16; off <<= 1) sse += __shfl_xor(sse, off, kWave);
    if (lane == 0) P[kNParam] = sse;
}

// Sums the per-wave partials in a fixed order.  With Adam (step > 0) it
// updates the FP32 master weights (Kingma & Ba, bias-corrected); otherwise it
// writes the gradient to `grad`.  out[0] = mean squared error of the batch.
// Sums the per-wave partials of every parameter (and of the loss) in FP64
// and applies Adam.  One lane per parameter, kRedWaves waves per block: wave
// w adds the partials w, w + kRedWaves, ... in that order, then the first
// wave adds the waves' sums in wave order, so the result depends only on
// the number of partials, not on timing.
constexpr int kRedWaves = 16;
__global__ __launch_bounds__(kRedWaves * kWave) void k_mlp_reduce(const float* __restrict__ part, int32_t nparts,
                                                                  int64_t batch, float* __restrict__ params,
                                                                  float* __restrict__ m, float* __restrict__ v,
                                                                  float* __restrict__ grad, int32_t step,
                                                                  double lr, double* __restrict__ out) {
    __shared__ double lds[kRedWaves][kWave];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int p = blockIdx.x * kWave + lane;
    double sw = 0.0;
    if (p <= kNParam) {
#pragma unroll 8
        for (int q = w; q < nparts; q += kRedWaves) sw += (double)part[(int64_t)q * (kNParam + 1) + p];
    }
    lds[w][lane] = sw;
    __syncthreads();
    if (w != 0 || p > kNParam) return;
    double s = 0.0;
    for (int k = 0; k < kRedWaves; ++k) s += lds[k][lane];
    if (p == kNParam) {
        out[0] = s / (double)batch;
        return;
    }
    if (step <= 0) {
        grad[p] = (float)s;
        return;
    }
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double mm = b1 * (double)m[p] + (1.0 - b1) * s;
    const double vv = b2 * (double)v[p] + (1.0 - b2) * s * s;
    const double mh = mm / (1.0 - pow(b1, (double)step));
    const double vh = vv / (1.0 - pow(b2, (double)step));
    params[p] = (float)((double)params[p] - lr * mh / (sqrt(vh) + eps));
    m[p] = (float)mm;
    v[p] = (float)vv;
}

}  // namespace mlp
}  // namespace sph

using namespace sph;
using namespace sph::mlp;

static int32_t tiles_per_wave(int64_t n, int32_t* grid) {
    const int64_t tiles = ceil_div(n, 16);
    int64_t waves = std::min<int64_t>(ceil_div(tiles, 4), 8192);
    if (waves < 1) waves = 1;
    const int64_t blocks = ceil_div(waves, kWaves);
    *grid = (int32_t)blocks;
    return (int32_t)ceil_div(tiles, blocks * kWaves);
}

sph_status sph::mlp::forward(sph_ctx* ctx, const float* samples, int64_t n, const float* params, float* out) {
    if (n == 0) return SPH_OK;
    // several tiles per wave: each wave loads its 32 weight fragments once
    const int64_t waves = std::min<int64_t>(ceil_div(ceil_div(n, (int64_t)16), 4), 8192);
    const int32_t grid = (int32_t)std::max<int64_t>(ceil_div(waves, (int64_t)kWaves), 1);
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(kThreads), 0, ctx->stream, samples, n, params, out);
    SPH_LAUNCHED("k_mlp_infer");
    return SPH_OK;
}

extern "C" sph_status sph_mlp_forward(sph_ctx* ctx, const float* samples, int64_t n, const float* params,
                                      float* out) {
    if (!ctx) return SPH_E_ARG;
    if (!samples || !params || !out || n < 0) return ctx->fail(SPH_E_ARG, "mlp_forward: bad argument");
    if (reinterpret_cast<uintptr_t>(samples) % 16 || reinterpret_cast<uintptr_t>(out) % 16)
        return ctx->fail(SPH_E_ARG, "mlp_forward: samples and out must be 16-byte aligned");
    return sph::mlp::forward(ctx, samples, n, params, out);
}

static sph_status train_or_grad(sph_ctx* ctx, const float* samples, const int32_t* idx, int64_t batch,
                                float* params, float* m, float* v, float* grad, int32_t step, double lr,
                                double* loss) {
    int32_t grid = 0;
    const int32_t tpw = tiles_per_wave(batch, &grid);
    const int64_t nparts = (int64_t)grid * kWaves;
    float* part = nullptr;
    double* out = nullptr;
    SPH_TRY(ctx->ensure_t(kMlpPart, (size_t)nparts * (kNParam + 1), &part));
    SPH_TRY(ctx->ensure_t(kMlpOut, 1, &out));
    hipLaunchKernelGGL(k_mlp_train, dim3(grid), dim3(kThreads), 0, ctx->stream, samples, idx, batch, params, part,
                       tpw);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)ceil_div(kNParam + 1, kWave)), dim3(kRedWaves * kWave), 0,
                       ctx->stream, part,
                       (int32_t)nparts, batch, params, m, v, grad, step, lr, out);
    SPH_LAUNCHED("k_mlp_train/k_mlp_reduce");
    if (loss) {
        SPH_HIP(hipMemcpyAsync(loss, out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        SPH_HIP(hipStreamSynchronize(ctx->stream));
    }
    return SPH_OK;
}

extern "C" sph_status sph_mlp_grad(sph_ctx* ctx, const float* samples, const int32_t* idx, int64_t batch,
                                   const float* params, float* grad, double* loss) {
    if (!ctx) return SPH_E_ARG;
    if (!samples || !idx || !params || !grad || batch < 1) return ctx->fail(SPH_E_ARG, "mlp_grad: bad argument");
    return train_or_grad(ctx, samples, idx, batch, const_cast<float*>(params), nullptr, nullptr, grad, 0, 0.0, loss);
}

extern "C" sph_status sph_mlp_train_step(sph_ctx* ctx, const float* samples, const int32_t* idx, int64_t batch,
                                         float* params, float* adam_m, float* adam_v, int32_t step, double lr,
                                         double* loss) {
    if (!ctx) return SPH_E_ARG;
    if (!samples || !idx || !params || !adam_m || !adam_v || batch < 1 || step < 1 || !(lr > 0.0))
        return ctx->fail(SPH_E_ARG, "mlp_train_step: bad argument");
    return train_or_grad(ctx, samples, idx, batch, params, adam_m, adam_v, nullptr, step, lr, loss);
}
