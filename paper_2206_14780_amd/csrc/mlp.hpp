// Layout of the warm-start MLP's parameters and samples (shared by the MLP
// kernels and the solver's warm-start path).
#pragma once

#include "sph_internal.hpp"

namespace sph {
namespace mlp {

constexpr int kIn = 4, kH = 64, kOut = 3;
// flat FP32 parameter vector: W1 [4][64], b1, W2 [64][64], b2, W3 [64][64], b3, W4 [64][3], b4
constexpr int kOW1 = 0;
constexpr int kOB1 = kOW1 + kIn * kH;
constexpr int kOW2 = kOB1 + kH;
constexpr int kOB2 = kOW2 + kH * kH;
constexpr int kOW3 = kOB2 + kH;
constexpr int kOB3 = kOW3 + kH * kH;
constexpr int kOW4 = kOB3 + kH;
constexpr int kOB4 = kOW4 + kH * kOut;
constexpr int kNParam = kOB4 + kOut;
static_assert(kNParam == SPH_MLP_NPARAM, "parameter count");
// one sample: features x[4], basis B[3], target t
constexpr int kSample = SPH_MLP_SAMPLE;

// out[s] = (o0, o1, o2, pred) of samples [0, n) on the context stream.
sph_status forward(sph_ctx* ctx, const float* samples, int64_t n, const float* params, float* out);

}  // namespace mlp

// Layout of the learned-start record in device memory (doubles).
constexpr int kWiRrL = 0;    // [3] true r.r of the learned guess
constexpr int kWiRrP = 3;    // [3] true r.r of the plain start
constexpr int kWiUse = 6;    // [3] 1.0 where the learned guess is kept
constexpr int kWiU = 9;      // U
constexpr int kWiLogNu = 10; // mean of log10 nu over fluid rows
constexpr int kWiSize = 16;

// Operator data the learned start needs (cell order).
template <typename T>
struct WarmOp {
    const sph_nbr* nb;
    PartView pv;
    OpParams op;
    int32_t mode;           // SPH_OP_CACHED / SPH_OP_ONTHEFLY
    const Sell<T>* sell;    // cached mode
    const double* diag64;   // D = A_rr
};

// Optional output of the feature pass (cached operator only): the residual
// b64 - A u of the start x0 = u (T, cell order AoS) and 3 partials of its
// r.r per block of the pass (kWarmFeatBlocks at most).
template <typename T>
struct PlainResidual {
    const double* b64;
    T* r;
    double* part;
};
constexpr int kWarmFeatBlocks = 2048;

// U and the samples of every row: orig_order = 1 writes sample 3 perm[r] + c
// (caller order), 0 writes 3 r + c (cell order).  rhs: caller order, of the
// caller's precision C; u: cell order, AoS; tgt: caller order FP64 or null.
// info: kWiSize doubles.
template <typename T, typename C>
sph_status warm_samples(sph_ctx* ctx, const WarmOp<T>& w, const void* const rhs[3], const C* u,
                        const double* const tgt[3], int32_t orig_order, float* samples, double* info,
                        const PlainResidual<T>* pr);
// Partials (3 per block, nblk blocks) of b64 . b64 (true r.r of the zero start).
sph_status warm_zero_rr(sph_ctx* ctx, int64_t n, int32_t nblk, const double* b64, double* part);
// Per-component choice between the learned start (xl, residual rl) and the
// plain start (x, residual r0 if plain_given, else b) by their true r.r
// partials pl, pp (3 per part); x and r0 receive the chosen start.
template <typename T, typename X>
sph_status warm_select(sph_ctx* ctx, int64_t n, int32_t grid, int32_t block, const double* pl, int32_t nl,
                       const double* pp, int32_t np, int32_t plain_given, X* x, const T* xl, const T* rl,
                       const T* b, T* r0, double* info);
// The learned guess (cell order, AoS) into x; rhs of the caller's precision C.
template <typename T, typename C>
sph_status warm_learned(sph_ctx* ctx, const WarmOp<T>& w, const void* const rhs[3], const C* u,
                        const float* params, T* x, double* info, const PlainResidual<T>* pr);

}  // namespace sph
