// Operator kernels y = A x, optionally fused with the inner products the
// solver needs from the same pass (the paper's gemv plus dot products,
// appendix "Implementation notes").
#pragma once

#include <cmath>

#include "sph_device.hpp"

namespace sph {

// Inner products produced per block alongside y = A x:
//   kDotA1     3 partials: w . y            (delta = r0hat . A p)
//   kDotA2     6 partials: x . y, y . y     (r* . A r*,  A r* . A r*)
//   kDotA2Std  9 partials: as kDotA2 plus x . x (textbook half-step check)
//   kDotResid  3 partials: y . y with y = b - A x evaluated in FP64 with the
//              FP64-accurate coefficients (true residual)
//   kDotCG     3 partials: <x, y>_D = sum_i D_i x_i y_i, the CG's p . A p in
//              the Jacobi-weighted inner product (D from the FP64 argument;
//              null: D = 1)
enum DotMode { kDotNone = 0, kDotA1 = 1, kDotA2 = 2, kDotA2Std = 3, kDotResid = 4, kDotCG = 5 };

template <int MODE>
struct DotK {
    static constexpr int K = MODE == kDotA1 ? 3 : MODE == kDotA2 ? 6 : MODE == kDotA2Std ? 9
                             : MODE == kDotResid ? 3 : MODE == kDotCG ? 3 : 1;
};

// KH: the paper's single precision (products rounded to FP32, compensated
// FP32 sums; see kahan_add), else FP64 products and sums.
template <typename T, int MODE, bool KH = false>
__device__ inline void accumulate_dots(double (&acc)[DotK<MODE>::K], float (&cmp)[DotK<MODE>::K], V3<T> xs,
                                       V3<T> yv, V3<T> wv, double dw = 1.0) {
    if constexpr (MODE == kDotCG) {
        dot_add_w<KH>(acc[0], cmp[0], dw, (double)xs.x, (double)yv.x);
        dot_add_w<KH>(acc[1], cmp[1], dw, (double)xs.y, (double)yv.y);
        dot_add_w<KH>(acc[2], cmp[2], dw, (double)xs.z, (double)yv.z);
    } else if constexpr (MODE == kDotA1) {
        dot_add<KH>(acc[0], cmp[0], (double)wv.x, (double)yv.x);
        dot_add<KH>(acc[1], cmp[1], (double)wv.y, (double)yv.y);
        dot_add<KH>(acc[2], cmp[2], (double)wv.z, (double)yv.z);
    } else if constexpr (MODE == kDotA2 || MODE == kDotA2Std) {
        dot_add<KH>(acc[0], cmp[0], (double)xs.x, (double)yv.x);
        dot_add<KH>(acc[1], cmp[1], (double)xs.y, (double)yv.y);
        dot_add<KH>(acc[2], cmp[2], (double)xs.z, (double)yv.z);
        dot_add<KH>(acc[3], cmp[3], (double)yv.x, (double)yv.x);
        dot_add<KH>(acc[4], cmp[4], (double)yv.y, (double)yv.y);
        dot_add<KH>(acc[5], cmp[5], (double)yv.z, (double)yv.z);
        if constexpr (MODE == kDotA2Std) {
            dot_add<KH>(acc[6], cmp[6], (double)xs.x, (double)xs.x);
            dot_add<KH>(acc[7], cmp[7], (double)xs.y, (double)xs.y);
            dot_add<KH>(acc[8], cmp[8], (double)xs.z, (double)xs.z);
        }
    }
}


// Column jump held in the coefficient bits of an escape slot.
__device__ inline int32_t jump_bits(float w) { return __float_as_int(w); }
__device__ inline int32_t jump_bits(double w) { return (int32_t)__double_as_longlong(w); }

// Entries per software-pipelined group: 16 for the FP32 operator (more
// loads in flight), 8 where FP64 values or the FP64-accurate residual would
// not fit the registers.
template <typename T, bool RES>
constexpr int group_of() { return sizeof(T) == 4 && !RES ? 16 : 8; }

// Raw slots of one group (zero beyond the row's width): a lane's kPack
// adjacent slots come in one vector load each for the coefficients, the
// column steps and (residual) the low parts.  Widths and groups are
// multiples of kPack, so a pack is either wholly inside the row or beyond it.
template <typename T, int P>
struct Pack {
    typedef T v __attribute__((ext_vector_type(P)));
};
template <typename T>
struct Pack<T, 1> {
    typedef T v;
};

template <typename T, int P>
__device__ inline T pack_elem(const typename Pack<T, P>::v& v, int e) {
    if constexpr (P == 1) return v;
    else return v[e];
}

template <typename T, bool RES>
__device__ inline void sell_group(const Sell<T>& A, int64_t base, int32_t width, int32_t k0,
                                  T (&w)[group_of<T, RES>()], uint16_t (&d)[group_of<T, RES>()],
                                  double (&l)[group_of<T, RES>()]) {
    constexpr int kGroup = group_of<T, RES>();
    constexpr int P = pack_of<T>();
    static_assert(kGroup % P == 0, "whole packs per group");
#pragma unroll
    for (int q = 0; q < kGroup / P; ++q) {
        const int32_t k = k0 + q * P;
        if (k < width) {
            const int64_t i = slot_of<T>(base, k);
            // read once per launch: non-temporal, so the stream does not
            // evict the x values that the gathers reuse from L2
            const typename Pack<T, P>::v wv =
                __builtin_nontemporal_load(reinterpret_cast<const typename Pack<T, P>::v*>(A.coef + i));
            const typename Pack<uint16_t, P>::v dv =
                __builtin_nontemporal_load(reinterpret_cast<const typename Pack<uint16_t, P>::v*>(A.dcol + i));
#pragma unroll
            for (int e = 0; e < P; ++e) {
                w[q * P + e] = pack_elem<T, P>(wv, e);
                d[q * P + e] = pack_elem<uint16_t, P>(dv, e);
            }
            if constexpr (RES && sizeof(T) == 4) {
                const typename Pack<float, P>::v lv =
                    __builtin_nontemporal_load(reinterpret_cast<const typename Pack<float, P>::v*>(A.lo + i));
#pragma unroll
                for (int e = 0; e < P; ++e) l[q * P + e] = (double)pack_elem<float, P>(lv, e);
            } else {
#pragma unroll
                for (int e = 0; e < P; ++e) l[q * P + e] = 0.0;
            }
        } else {
#pragma unroll
            for (int e = 0; e < P; ++e) {
                w[q * P + e] = T(0);
                d[q * P + e] = 0;
                l[q * P + e] = 0.0;
            }
        }
    }
}

// sum_k coef[r,k] (x[col[r,k]] - x_r) for the row of this lane (the operator's
// difference form: rounding scales with the local variation of x, not with x,
// so smooth fields keep their accuracy in FP32).  `base` is the lane's first
// slot, `width` the slice width (uniform across the wave).  The loop is
// software-pipelined: the gathers of group g are issued before the slot loads
// of group g + 1, so the L2 latency of the gathers and the HBM latency of the
// matrix stream overlap; the column steps of a group are summed before its
// gathers.  RES accumulates in FP64 with the FP64-accurate coefficients; x
// may then be of another precision XT than the matrix (an FP64 solution
// under an FP32 operator).
template <typename T, bool RES, typename ACC, typename XT = T>
__device__ inline void sell_row(const Sell<T>& A, int64_t base, int32_t width, int32_t row,
                                const XT* __restrict__ x, const V3<XT>& xs, ACC& a0, ACC& a1, ACC& a2) {
    constexpr int kGroup = group_of<T, RES>();
    int32_t col = A.c0[row];
    T rw[kGroup];
    uint16_t rd[kGroup];
    double rl[kGroup];
    sell_group<T, RES>(A, base, width, 0, rw, rd, rl);
    for (int32_t k0 = 0; k0 < width; k0 += kGroup) {
        int32_t cc[kGroup];
        T cw[kGroup];
        double cl[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const bool esc = rd[u] == kEscape;
            col += esc ? jump_bits(rw[u]) : (int32_t)rd[u];
            cw[u] = esc ? T(0) : rw[u];
            cl[u] = esc ? 0.0 : rl[u];
            // escape and padding slots (zero weight) gather the lane's own
            // row: the 64 lanes' own rows share a few cache lines, where
            // their last columns would scatter over many
            cc[u] = (cw[u] == T(0) && cl[u] == 0.0) ? row : col;
        }
        V3<XT> xv[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) xv[u] = ld3(x, cc[u]);
        sell_group<T, RES>(A, base, width, k0 + kGroup, rw, rd, rl);
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            if constexpr (RES) {
                const double w = (double)cw[u] + cl[u];
                a0 += w * ((double)xv[u].x - (double)xs.x);
                a1 += w * ((double)xv[u].y - (double)xs.y);
                a2 += w * ((double)xv[u].z - (double)xs.z);
            } else {
                a0 = fma_t(cw[u], xv[u].x - xs.x, a0);
                a1 = fma_t(cw[u], xv[u].y - xs.y, a1);
                a2 = fma_t(cw[u], xv[u].z - xs.z, a2);
            }
        }
    }
}

// The paper's single-precision gemv of one row: y_r = A_rr x_r + sum_k
// coef[r,k] x[col[r,k]] with every product rounded to FP32 and the terms
// added in slot order by Kahan's compensated summation (zero-weight escape
// and padding slots add nothing).  d: the plain diagonal A_rr.
__device__ inline void sell_row_kahan(const Sell<float>& A, int64_t base, int32_t width, int32_t row,
                                      const float* __restrict__ x, const V3<float>& xs, float d, V3<float>& y) {
    constexpr int kGroup = group_of<float, false>();
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    kahan_add(s0, c0, d * xs.x);
    kahan_add(s1, c1, d * xs.y);
    kahan_add(s2, c2, d * xs.z);
    int32_t col = A.c0[row];
    float rw[kGroup];
    uint16_t rd[kGroup];
    double rl[kGroup];
    sell_group<float, false>(A, base, width, 0, rw, rd, rl);
    for (int32_t k0 = 0; k0 < width; k0 += kGroup) {
        int32_t cc[kGroup];
        float cw[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const bool esc = rd[u] == kEscape;
            col += esc ? jump_bits(rw[u]) : (int32_t)rd[u];
            cw[u] = esc ? 0.f : rw[u];
            cc[u] = cw[u] == 0.f ? row : col;
        }
        V3<float> xv[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) xv[u] = ld3(x, cc[u]);
        sell_group<float, false>(A, base, width, k0 + kGroup, rw, rd, rl);
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            if (cw[u] != 0.f) {
                kahan_add(s0, c0, cw[u] * xv[u].x);
                kahan_add(s1, c1, cw[u] * xv[u].y);
                kahan_add(s2, c2, cw[u] * xv[u].z);
            }
        }
    }
    y = V3<float>{s0, s1, s2};
}

// Cached operator: y_r = rs_r x_r + sum_k coef[r,k] (x[col[r,k]] - x_r).
// One wavefront per 64-row slice; each block takes a contiguous range of
// slices (XCD-aware order) and its waves interleave over it.  With kDotResid
// the kernel writes y = b64 - A x (FP64-accurate, rounded to T) instead, and
// x may be held in another precision XT; with kDotCG, b64 holds the weights
// D of the inner product.
//
// KH (T = float only): the paper's single precision: the row in plain form
// with compensated FP32 sums (sell_row_kahan, A.dg the plain diagonal) and
// the inner products of FP32 products with compensated FP32 sums.
template <typename T, int MODE, typename XT = T, bool KH = false>
__global__ __launch_bounds__(kApplyMaxBlock) void k_apply_sell(const int32_t* __restrict__ halt, int64_t n, Sell<T> A,
                                                          const XT* __restrict__ x, T* __restrict__ y,
                                                          const T* __restrict__ w, const double* __restrict__ b64,
                                                          double* __restrict__ part) {
    if (halt && *halt) return;
    constexpr int K = DotK<MODE>::K;
    constexpr bool RES = MODE == kDotResid;
    static_assert(!KH || (sizeof(T) == 4 && !RES), "single-precision arithmetic: FP32 operator, not the residual");
    __shared__ double lds[(KH ? 2 : 1) * K * kMaxWaves];
    double acc[K];
    float cmp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[k] = 0.0;
        cmp[k] = 0.f;
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t spb = ceil_div(A.nslices, (int64_t)gridDim.x);
    const int64_t s0 = bid * spb;
    const int64_t s1 = min(s0 + spb, A.nslices);
    for (int64_t s = s0 + wid; s < s1; s += nw) {
        const int64_t row = s * kWave + lane;
        if (row >= n) continue;
        const int64_t base = lane_base<T>(A.sl_ptr[s], lane);
        const int32_t width = (int32_t)((A.sl_ptr[s + 1] - A.sl_ptr[s]) / kWave);
        const V3<XT> xs = ld3(x, row);
        if constexpr (RES) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            sell_row<T, true, double, XT>(A, base, width, (int32_t)row, x, xs, a0, a1, a2);
            const double d = A.rs64[row];
            const V3<double> bb = ld3(b64, row);
            const double r0 = bb.x - (d * (double)xs.x + a0);
            const double r1 = bb.y - (d * (double)xs.y + a1);
            const double r2 = bb.z - (d * (double)xs.z + a2);
            acc[0] += r0 * r0;
            acc[1] += r1 * r1;
            acc[2] += r2 * r2;
            st3(y, row, V3<T>{(T)r0, (T)r1, (T)r2});
        } else {
            V3<T> yv;
            if constexpr (KH) {
                sell_row_kahan(A, base, width, (int32_t)row, x, xs, A.dg[row], yv);
            } else {
                T a0 = T(0), a1 = T(0), a2 = T(0);
                sell_row<T, false>(A, base, width, (int32_t)row, x, xs, a0, a1, a2);
                const T d = A.dg[row];
                yv.x = fma_t(d, xs.x, a0);
                yv.y = fma_t(d, xs.y, a1);
                yv.z = fma_t(d, xs.z, a2);
            }
            st3(y, row, yv);
            if constexpr (MODE != kDotNone) {
                V3<T> wv{};
                if constexpr (MODE == kDotA1) wv = ld3(w, row);
                double dw = 1.0;
                if constexpr (MODE == kDotCG) dw = b64 ? b64[row] : 1.0;
                accumulate_dots<T, MODE, KH>(acc, cmp, xs, yv, wv, dw);
            }
        }
    }
    if constexpr (MODE != kDotNone) write_partials_kh<K, KH>(acc, cmp, lds, part);
}

// One row of the operator evaluated from positions in FP64 (the paper's
// matrix-free gemv): returns (A x)_b, or (D^-1 A x)_b with Jacobi.
template <typename T>
__device__ inline void row_apply_otf(const NbrView& nv, const PartView& pv, const OpParams& op,
                                     const T* __restrict__ x, int32_t b, double (&y)[3]) {
    const V3<T> xb = ld3(x, b);
    y[0] = (double)xb.x;
    y[1] = (double)xb.y;
    y[2] = (double)xb.z;
    if (pv.type[b] == SPH_FLUID) {
        double sw = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for_each_neighbor(nv, b, [&](int32_t a, double r2) {
            const double wgt = pair_w(pv, nv.g, op.avg, b, a, r2);
            const V3<T> xa = ld3(x, a);
            sw += wgt;
            s0 += wgt * (double)xa.x;
            s1 += wgt * (double)xa.y;
            s2 += wgt * (double)xa.z;
        });
        const double diag = 1.0 + op.dt * sw;
        y[0] = diag * y[0] - op.dt * s0;
        y[1] = diag * y[1] - op.dt * s1;
        y[2] = diag * y[2] - op.dt * s2;
        if (op.jacobi) {
            y[0] /= diag;
            y[1] /= diag;
            y[2] /= diag;
        }
    } else if (op.wall == SPH_WALL_DUMMY) {
        double sW = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for_each_neighbor(nv, b, [&](int32_t a, double r2) {
            if (pv.type[a] != SPH_FLUID) return;
            const double W = pair_W(nv.g, r2);
            const V3<T> xa = ld3(x, a);
            sW += W;
            s0 += W * (double)xa.x;
            s1 += W * (double)xa.y;
            s2 += W * (double)xa.z;
        });
        if (sW > 0.0) {
            y[0] += s0 / sW;
            y[1] += s1 / sW;
            y[2] += s2 / sW;
        }
    }
}

// On-the-fly operator over rows in cell order; with kDotResid it writes
// y = b64 - A x instead (FP64 residual rounded to T) and its squared norm,
// x then being of precision XT; with kDotCG, b64 holds the weights D.
template <typename T, int MODE, typename XT = T>
__global__ __launch_bounds__(kApplyMaxBlock) void k_apply_otf(const int32_t* __restrict__ halt, NbrView nv, PartView pv,
                                                         OpParams op, const XT* __restrict__ x, T* __restrict__ y,
                                                         const T* __restrict__ w, const double* __restrict__ b64,
                                                         double* __restrict__ part) {
    if (halt && *halt) return;
    constexpr int K = DotK<MODE>::K;
    __shared__ double lds[K * kMaxWaves];
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t rpb = ceil_div(nv.n, (int64_t)gridDim.x);
    const int64_t r0 = bid * rpb;
    const int64_t r1 = min(r0 + rpb, nv.n);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        double yv[3];
        row_apply_otf<XT>(nv, pv, op, x, (int32_t)r, yv);
        if constexpr (MODE == kDotResid) {
            const V3<double> bb = ld3(b64, r);
            yv[0] = bb.x - yv[0];
            yv[1] = bb.y - yv[1];
            yv[2] = bb.z - yv[2];
            acc[0] += yv[0] * yv[0];
            acc[1] += yv[1] * yv[1];
            acc[2] += yv[2] * yv[2];
        }
        V3<T> out;
        out.x = (T)yv[0];
        out.y = (T)yv[1];
        out.z = (T)yv[2];
        st3(y, r, out);
        if constexpr (MODE != kDotNone && MODE != kDotResid) {
            V3<T> wv{};
            if constexpr (MODE == kDotA1) wv = ld3(w, r);
            double dw = 1.0;
            if constexpr (MODE == kDotCG) dw = b64 ? b64[r] : 1.0;
            float cmp[K];
            accumulate_dots<T, MODE>(acc, cmp, ld3(x, r), out, wv, dw);
        }
    }
    if constexpr (MODE != kDotNone) write_partials<K>(acc, lds, part);
}

}  // namespace sph
