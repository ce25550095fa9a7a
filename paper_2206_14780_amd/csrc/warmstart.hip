// Learned initial guess: features of the current state, the MLP's start on
// fluid rows, exact dummy-wall rows, and the per-component choice between
// the learned and the plain start by FP64 true residual.  Not part of the
// paper, which names better initial guesses as future work (Sections
// "Conclusions and future work" and "Implementation notes").
//
// One sample per fluid row r and component c (wall rows: all zero):
//   d = (u - A u) / A_rr = -(1/A_rr) sum_k A_rk (u_k - u_r)   (one Jacobi
//       correction of u: the viscous increment scaled by the row's diagonal)
//   x = (u_c / U, d_c / U, log10 nu_r - L, log10(dt nu_r / h^2)),  nu = mu / rho
//   B = (b_c / U, u_c / U, d_c / U),  t = V_c / U (training only)
// with U the RMS of b over fluid rows and components (1 if that is 0) and L
// the mean of log10 nu over fluid rows: the viscosity enters relative to the
// system's geometric-mean viscosity (scale-free), its magnitude through the
// stiffness dt nu / h^2.
#include <algorithm>
#include <cmath>

#include "mlp.hpp"
#include "operator_kernels.hpp"

namespace sph {

using mlp::kSample;

namespace {

constexpr int kStatBlocks = 256;
constexpr unsigned kFeatBlocks = kWarmFeatBlocks;  // grid of the cached-operator feature kernel

template <typename C>
struct Rhs {
    const int32_t* perm;  // cell -> caller order
    const C* b[3];        // caller order, caller precision
    __device__ double at(int64_t r, int c) const { return (double)b[c][perm[r]]; }
};

// Partial sums over fluid rows of b.b, of the row count and of log10 nu, in
// the caller's order (b read contiguously; type, mu and rho through iperm).
template <typename C>
__global__ __launch_bounds__(kBlock) void k_warm_stats(int64_t n, Rhs<C> rhs, const int32_t* __restrict__ iperm,
                                                       PartView pv, double* __restrict__ part) {
    __shared__ double lds[3 * kMaxWaves];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = iperm[i];
        if (pv.type[r] != SPH_FLUID) continue;
        for (int c = 0; c < 3; ++c) {
            const double v = (double)rhs.b[c][i];
            acc[0] += v * v;
        }
        acc[1] += 1.0;
        acc[2] += log10(pv.mu[r] / pv.rho[r]);
    }
    write_partials<3>(acc, lds, part);
}

__global__ __launch_bounds__(kBlock) void k_warm_scale(const double* __restrict__ part, int nblk,
                                                       double* __restrict__ info) {
    __shared__ double lds[3 * kMaxWaves];
    double s[3];
    reduce_partials<3>(part, nblk, s, lds);
    if (threadIdx.x == 0) {
        double U = s[1] > 0.0 ? sqrt(s[0] / (3.0 * s[1])) : 0.0;
        if (!(U > 0.0) || !finite_d(U)) U = 1.0;
        info[kWiU] = U;
        const double L = s[1] > 0.0 ? s[2] / s[1] : 0.0;
        info[kWiLogNu] = finite_d(L) ? L : 0.0;
    }
}

// Writes the 3 samples of row r given d.
template <typename C>
__device__ inline void warm_write(int64_t r, const Rhs<C>& rhs, const V3<C>& u, const double (&d)[3],
                                  const PartView& pv, double dt, double h, double U, double lognu_mean,
                                  const double* const* tgt, float* __restrict__ out) {
    const double nu = pv.mu[r] / pv.rho[r];
    const float f2 = (float)(log10(nu) - lognu_mean);
    const float f3 = (float)log10(dt * nu / (h * h));
    const double uu[3] = {(double)u.x, (double)u.y, (double)u.z};
    for (int c = 0; c < 3; ++c) {
        float4* o = reinterpret_cast<float4*>(out + c * kSample);  // rows of 8 floats, 32-byte aligned
        const double uc = uu[c] / U, ic = d[c] / U;
        o[0] = float4{(float)uc, (float)ic, f2, f3};
        o[1] = float4{(float)(rhs.at(r, c) / U), (float)uc, (float)ic,
                      tgt ? (float)(tgt[c][rhs.perm[r]] / U) : 0.f};
    }
}

template <typename T, typename C>
struct FeatArgs {
    int64_t n;
    Rhs<C> rhs;
    const C* u;              // cell order, AoS, caller precision
    PartView pv;
    double dt, h;
    const double* diag64;    // D = A_rr
    int32_t jacobi;
    const double* info;      // U at kWiU
    const double* tgt[3];    // caller order, or null
    int32_t has_tgt;
    int32_t orig_order;
    float* samples;
    // optional (cached operator): the FP64-accurate residual b64 - A u of the
    // start x0 = u, rounded to T, and per-block partials of its r.r
    const double* b64;
    T* rplain;
    double* part;
};

template <typename T, typename C>
__device__ inline float* sample_row(const FeatArgs<T, C>& a, int64_t r) {
    const int64_t k = a.orig_order ? (int64_t)a.rhs.perm[r] : r;
    return a.samples + k * 3 * kSample;
}

__device__ inline void zero_row(float* o) {
    float4* q = reinterpret_cast<float4*>(o);
    for (int k = 0; k < 3 * kSample / 4; ++k) q[k] = float4{0.f, 0.f, 0.f, 0.f};
}

// Cached matrix: d = -sum_k c_k (u_k - u_r) with c = A_rk / D (Jacobi
// scaled), or -(1/D) sum_k c_k (u_k - u_r) with c = A_rk.  The same FP64
// sum gives the residual of x0 = u, b - (rs u + sum_k c_k (u_k - u_r)), on
// every row when a.rplain is set (grid-stride, fixed grid).
template <typename T, typename C>
__global__ __launch_bounds__(kBlock) void k_warm_feat_sell(FeatArgs<T, C> a, Sell<T> A) {
    __shared__ double lds[3 * kMaxWaves];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.n;
         r += (int64_t)gridDim.x * blockDim.x) {
        float* o = sample_row(a, r);
        const bool fluid = a.pv.type[r] == SPH_FLUID;
        if (!fluid) zero_row(o);
        if (!fluid && !a.rplain) continue;
        const int64_t s = r / kWave;
        const int64_t base = lane_base<T>(A.sl_ptr[s], r % kWave);
        const int32_t width = (int32_t)((A.sl_ptr[s + 1] - A.sl_ptr[s]) / kWave);
        const V3<C> us = ld3(a.u, r);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        sell_row<T, true, double, C>(A, base, width, (int32_t)r, a.u, us, s0, s1, s2);
        if (a.rplain) {
            const double rs = A.rs64[r];
            const V3<double> bb = ld3(a.b64, r);
            const double q0 = bb.x - (rs * (double)us.x + s0);
            const double q1 = bb.y - (rs * (double)us.y + s1);
            const double q2 = bb.z - (rs * (double)us.z + s2);
            acc[0] += q0 * q0;
            acc[1] += q1 * q1;
            acc[2] += q2 * q2;
            st3(a.rplain, r, V3<T>{(T)q0, (T)q1, (T)q2});
        }
        if (!fluid) continue;
        double d[3] = {-s0, -s1, -s2};
        if (!a.jacobi) {
            const double D = a.diag64[r];
            for (int c = 0; c < 3; ++c) d[c] /= D;
        }
        warm_write<C>(r, a.rhs, us, d, a.pv, a.dt, a.h, a.info[kWiU], a.info[kWiLogNu],
                      a.has_tgt ? a.tgt : nullptr, o);
    }
    if (a.rplain) write_partials<3>(acc, lds, a.part);
}

// On-the-fly operator: d = dt sum_a w_ra (u_a - u_r) / D.
template <typename T, typename C>
__global__ __launch_bounds__(kBlock) void k_warm_feat_otf(FeatArgs<T, C> a, NbrView nv, int32_t avg) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    float* o = sample_row(a, r);
    if (a.pv.type[r] != SPH_FLUID) {
        zero_row(o);
        return;
    }
    const V3<C> us = ld3(a.u, r);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for_each_neighbor(nv, (int32_t)r, [&](int32_t k, double r2) {
        const double w = pair_w(a.pv, nv.g, avg, (int32_t)r, k, r2);
        const V3<C> uk = ld3(a.u, k);
        s0 += w * ((double)uk.x - (double)us.x);
        s1 += w * ((double)uk.y - (double)us.y);
        s2 += w * ((double)uk.z - (double)us.z);
    });
    const double f = a.dt / a.diag64[r];
    const double d[3] = {f * s0, f * s1, f * s2};
    warm_write<C>(r, a.rhs, us, d, a.pv, a.dt, a.h, a.info[kWiU], a.info[kWiLogNu], a.has_tgt ? a.tgt : nullptr,
                  o);
}

// x = U pred on fluid rows, b on dynamic walls, 0 on dummy walls (filled next).
template <typename T, typename C>
__global__ __launch_bounds__(kBlock) void k_warm_x0(int64_t n, Rhs<C> rhs, const uint8_t* __restrict__ type,
                                                    int32_t wall, const float* __restrict__ mlp_out,
                                                    const double* __restrict__ info, T* __restrict__ x) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double v[3];
    if (type[r] == SPH_FLUID) {
        const double U = info[kWiU];
        for (int c = 0; c < 3; ++c) v[c] = U * (double)mlp_out[(3 * r + c) * 4 + 3];
    } else if (wall == SPH_WALL_DYNAMIC) {
        for (int c = 0; c < 3; ++c) v[c] = rhs.at(r, c);
    } else {
        v[0] = v[1] = v[2] = 0.0;
    }
    st3(x, r, V3<T>{(T)v[0], (T)v[1], (T)v[2]});
}

// Dummy wall rows: x_w = b_w - sum_a A_wa x_a (the stored entries of a dummy
// wall row are its fluid neighbours' normalised kernel values; D = 1 there).
template <typename T, typename C>
__global__ __launch_bounds__(kBlock) void k_warm_wall_sell(int64_t n, Rhs<C> rhs, const uint8_t* __restrict__ type,
                                                           Sell<T> A, T* __restrict__ x) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || type[r] == SPH_FLUID) return;
    const int64_t s = r / kWave;
    const int64_t base = lane_base<T>(A.sl_ptr[s], r % kWave);
    const int32_t width = (int32_t)((A.sl_ptr[s + 1] - A.sl_ptr[s]) / kWave);
    const V3<T> zero{T(0), T(0), T(0)};
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    sell_row<T, true>(A, base, width, (int32_t)r, x, zero, s0, s1, s2);
    st3(x, r, V3<T>{(T)(rhs.at(r, 0) - s0), (T)(rhs.at(r, 1) - s1), (T)(rhs.at(r, 2) - s2)});
}

template <typename T, typename C>
__global__ __launch_bounds__(kBlock) void k_warm_wall_otf(Rhs<C> rhs, NbrView nv, const uint8_t* __restrict__ type,
                                                          T* __restrict__ x) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nv.n || type[r] == SPH_FLUID) return;
    double sW = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for_each_neighbor(nv, (int32_t)r, [&](int32_t k, double r2) {
        if (type[k] != SPH_FLUID) return;
        const double W = pair_W(nv.g, r2);
        const V3<T> xk = ld3(x, k);
        sW += W;
        s0 += W * (double)xk.x;
        s1 += W * (double)xk.y;
        s2 += W * (double)xk.z;
    });
    double v[3] = {rhs.at(r, 0), rhs.at(r, 1), rhs.at(r, 2)};
    if (sW > 0.0) {
        v[0] -= s0 / sW;
        v[1] -= s1 / sW;
        v[2] -= s2 / sW;
    }
    st3(x, r, V3<T>{(T)v[0], (T)v[1], (T)v[2]});
}

template <typename T, typename C>
sph_status launch_features(sph_ctx* ctx, const WarmOp<T>& w, const FeatArgs<T, C>& a) {
    const unsigned grid = (unsigned)ceil_div(a.n, kBlock);
    if (w.mode == SPH_OP_CACHED)
        hipLaunchKernelGGL((k_warm_feat_sell<T, C>), dim3(std::min<unsigned>(grid, kFeatBlocks)), dim3(kBlock), 0,
                           ctx->stream, a, *w.sell);
    else
        hipLaunchKernelGGL((k_warm_feat_otf<T, C>), dim3(grid), dim3(kBlock), 0, ctx->stream, a, w.nb->view(),
                           w.op.avg);
    SPH_LAUNCHED("k_warm_feat");
    return SPH_OK;
}

template <typename C>
Rhs<C> make_rhs(const sph_nbr* nb, const void* const rhs[3]) {
    Rhs<C> r;
    r.perm = nb->perm;
    for (int c = 0; c < 3; ++c) r.b[c] = static_cast<const C*>(rhs[c]);
    return r;
}

// Partials (3 per block) of b.b, the true r.r of the zero start.
__global__ __launch_bounds__(kBlock) void k_warm_bb(int64_t n, const double* __restrict__ b64,
                                                    double* __restrict__ part) {
    __shared__ double lds[3 * kMaxWaves];
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t rpb = ceil_div(n, (int64_t)gridDim.x);
    const int64_t i0 = (int64_t)blockIdx.x * rpb, i1 = min(i0 + rpb, n);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const V3<double> b = ld3(b64, i);
        acc[0] += b.x * b.x;
        acc[1] += b.y * b.y;
        acc[2] += b.z * b.z;
    }
    write_partials<3>(acc, lds, part);
}

// Per component, keep the learned start (x <- xl, r0 <- rl) when its true
// r.r is smaller than the plain start's; otherwise r0 <- rp (plain start
// given) or b (zero start).  Every block reduces both sets of partials in
// the same fixed order, so all blocks take the same decision.
template <typename T, typename X>
__global__ __launch_bounds__(kMaxBlock) void k_warm_select(int64_t n, const double* __restrict__ pl, int nl,
                                                           const double* __restrict__ pp, int np,
                                                           int32_t plain_given, X* __restrict__ x,
                                                           const T* __restrict__ xl, const T* __restrict__ rl,
                                                           const T* __restrict__ b, T* __restrict__ r0,
                                                           double* __restrict__ info) {
    __shared__ double lds[3 * kMaxWaves];
    double rrl[3], rrp[3];
    reduce_partials<3>(pl, nl, rrl, lds);
    reduce_partials<3>(pp, np, rrp, lds);
    bool use[3];
    for (int c = 0; c < 3; ++c) use[c] = rrl[c] < rrp[c];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            info[kWiRrL + c] = rrl[c];
            info[kWiRrP + c] = rrp[c];
            info[kWiUse + c] = use[c] ? 1.0 : 0.0;
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        V3<X> xv = ld3(x, i);
        V3<T> rv = plain_given ? ld3(r0, i) : ld3(b, i);
        const V3<T> xlv = ld3(xl, i), rlv = ld3(rl, i);
        if (use[0]) { xv.x = (X)xlv.x; rv.x = rlv.x; }
        if (use[1]) { xv.y = (X)xlv.y; rv.y = rlv.y; }
        if (use[2]) { xv.z = (X)xlv.z; rv.z = rlv.z; }
        st3(x, i, xv);
        st3(r0, i, rv);
    }
}

}  // namespace

sph_status warm_zero_rr(sph_ctx* ctx, int64_t n, int32_t nblk, const double* b64, double* part) {
    hipLaunchKernelGGL(k_warm_bb, dim3(nblk), dim3(kBlock), 0, ctx->stream, n, b64, part);
    SPH_LAUNCHED("k_warm_bb");
    return SPH_OK;
}

template <typename T, typename X>
sph_status warm_select(sph_ctx* ctx, int64_t n, int32_t grid, int32_t block, const double* pl, int32_t nl,
                       const double* pp, int32_t np, int32_t plain_given, X* x, const T* xl, const T* rl,
                       const T* b, T* r0, double* info) {
    hipLaunchKernelGGL((k_warm_select<T, X>), dim3(grid), dim3(block), 0, ctx->stream, n, pl, nl, pp, np,
                       plain_given, x, xl, rl, b, r0, info);
    SPH_LAUNCHED("k_warm_select");
    return SPH_OK;
}

#define SPH_WARM_SELECT(T, X)                                                                                   \
    template sph_status warm_select<T, X>(sph_ctx*, int64_t, int32_t, int32_t, const double*, int32_t,          \
                                          const double*, int32_t, int32_t, X*, const T*, const T*, const T*, T*,   \
                                          double*);
SPH_WARM_SELECT(float, float)
SPH_WARM_SELECT(double, double)
SPH_WARM_SELECT(float, double)
#undef SPH_WARM_SELECT

template <typename T, typename C>
sph_status warm_samples(sph_ctx* ctx, const WarmOp<T>& w, const void* const rhs[3], const C* u,
                        const double* const tgt[3], int32_t orig_order, float* samples, double* info,
                        const PlainResidual<T>* pr) {
    const int64_t n = w.nb->n;
    double* part = nullptr;
    SPH_TRY(ctx->ensure_t(kWarmPart, 3 * kStatBlocks, &part));
    const Rhs<C> rb = make_rhs<C>(w.nb, rhs);
    const int sb = (int)std::min<int64_t>(kStatBlocks, std::max<int64_t>(1, ceil_div(n, kBlock)));
    hipLaunchKernelGGL(k_warm_stats<C>, dim3(sb), dim3(kBlock), 0, ctx->stream, n, rb, w.nb->iperm, w.pv, part);
    hipLaunchKernelGGL(k_warm_scale, dim3(1), dim3(kBlock), 0, ctx->stream, (const double*)part, sb, info);
    SPH_LAUNCHED("k_warm_stats/k_warm_scale");
    FeatArgs<T, C> a;
    a.n = n;
    a.rhs = rb;
    a.u = u;
    a.pv = w.pv;
    a.dt = w.op.dt;
    a.h = w.nb->g.h;
    a.diag64 = w.diag64;
    a.jacobi = w.op.jacobi;
    a.info = info;
    a.has_tgt = tgt != nullptr;
    for (int c = 0; c < 3; ++c) a.tgt[c] = tgt ? tgt[c] : nullptr;
    a.orig_order = orig_order;
    a.samples = samples;
    a.b64 = pr ? pr->b64 : nullptr;
    a.rplain = pr ? pr->r : nullptr;
    a.part = pr ? pr->part : nullptr;
    return launch_features<T, C>(ctx, w, a);
}

template <typename T, typename C>
sph_status warm_learned(sph_ctx* ctx, const WarmOp<T>& w, const void* const rhs[3], const C* u,
                        const float* params, T* x, double* info, const PlainResidual<T>* pr) {
    const int64_t n = w.nb->n;
    float *S = nullptr, *O = nullptr;
    SPH_TRY(ctx->ensure_t(kWarmS, (size_t)n * 3 * kSample, &S));
    SPH_TRY(ctx->ensure_t(kWarmO, (size_t)n * 3 * 4, &O));
    SPH_TRY((warm_samples<T, C>(ctx, w, rhs, u, nullptr, 0, S, info, pr)));
    SPH_TRY(mlp::forward(ctx, S, n * 3, params, O));
    const Rhs<C> rb = make_rhs<C>(w.nb, rhs);
    const unsigned grid = (unsigned)ceil_div(n, kBlock);
    hipLaunchKernelGGL((k_warm_x0<T, C>), dim3(grid), dim3(kBlock), 0, ctx->stream, n, rb, w.pv.type, w.op.wall,
                       (const float*)O, (const double*)info, x);
    if (w.op.wall == SPH_WALL_DUMMY) {
        if (w.mode == SPH_OP_CACHED)
            hipLaunchKernelGGL((k_warm_wall_sell<T, C>), dim3(grid), dim3(kBlock), 0, ctx->stream, n, rb, w.pv.type,
                               *w.sell, x);
        else
            hipLaunchKernelGGL((k_warm_wall_otf<T, C>), dim3(grid), dim3(kBlock), 0, ctx->stream, rb, w.nb->view(),
                               w.pv.type, x);
    }
    SPH_LAUNCHED("k_warm_x0/k_warm_wall");
    return SPH_OK;
}

#define SPH_WARM_INST(T, C)                                                                                    \
    template sph_status warm_samples<T, C>(sph_ctx*, const WarmOp<T>&, const void* const[3], const C*,           \
                                           const double* const[3], int32_t, float*, double*,                     \
                                           const PlainResidual<T>*);                                              \
    template sph_status warm_learned<T, C>(sph_ctx*, const WarmOp<T>&, const void* const[3], const C*,           \
                                           const float*, T*, double*, const PlainResidual<T>*);
SPH_WARM_INST(float, float)
SPH_WARM_INST(double, double)
SPH_WARM_INST(float, double)
#undef SPH_WARM_INST

}  // namespace sph

using namespace sph;

namespace {

template <typename T>
sph_status prepare(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, const sph_visc_params* v,
                   const void* const u[3], WarmOp<T>* w, Sell<T>* sell, T** ucell, double** info) {
    w->nb = nb;
    SPH_TRY(gather_props(ctx, nb, p, &w->pv));
    w->op = OpParams{v->dt, v->wall, v->avg, v->jacobi ? 1 : 0};
    w->op.f32cell = v->op_mode == SPH_OP_PAPER32 ? 1 : 0;
    w->mode = v->op_mode == SPH_OP_PAPER32 ? SPH_OP_CACHED : v->op_mode;
    w->sell = sell;
    if (w->mode == SPH_OP_CACHED)
        SPH_TRY(build_sell<T>(ctx, nb, w->pv, w->op, sell, &w->diag64));
    else
        SPH_TRY(row_diag64(ctx, nb, w->pv, w->op, &w->diag64));
    SPH_TRY(ctx->ensure_t(kApplyIn, (size_t)nb->n * 3, ucell));
    SPH_TRY(gather_vec3<T>(ctx, nb, u, *ucell));
    SPH_TRY(ctx->ensure_t(kWarmInfo, kWiSize, info));
    return SPH_OK;
}

sph_status check_common(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, const sph_visc_params* v,
                        int32_t prec, const void* const* u, const void* const* rhs, const char* who) {
    if (!nb || !u || !rhs) return ctx->fail(SPH_E_ARG, std::string(who) + ": null argument");
    if (nb->device != ctx->device) return ctx->fail(SPH_E_ARG, std::string(who) + ": handle of another device");
    for (int c = 0; c < 3; ++c)
        if (!u[c] || !rhs[c]) return ctx->fail(SPH_E_ARG, std::string(who) + ": null vector");
    SPH_TRY(check_particles(ctx, nb, p));
    return check_params(ctx, v, prec);
}

template <typename T>
sph_status warmstart_entry(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, const sph_visc_params* v,
                           const void* const u[3], const void* const rhs[3], const float* params,
                           void* const x0[3], double* U) {
    WarmOp<T> w;
    Sell<T> sell{};
    T* ucell = nullptr;
    double* info = nullptr;
    SPH_TRY(prepare<T>(ctx, nb, p, v, u, &w, &sell, &ucell, &info));
    T* x = nullptr;
    SPH_TRY(ctx->ensure_t(kApplyOut, (size_t)nb->n * 3, &x));
    SPH_TRY((warm_learned<T, T>(ctx, w, rhs, ucell, params, x, info, nullptr)));
    SPH_TRY(scatter_vec3<T>(ctx, nb, x, x0));
    if (U) {
        SPH_HIP(hipMemcpyAsync(U, info + kWiU, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        SPH_HIP(hipStreamSynchronize(ctx->stream));
    }
    return SPH_OK;
}

}  // namespace

extern "C" sph_status sph_mlp_samples(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p,
                                      const sph_visc_params* params, const double* const u[3],
                                      const double* const rhs[3], const double* const target[3], float* samples,
                                      double* U) {
    if (!ctx) return SPH_E_ARG;
    if (!samples) return ctx->fail(SPH_E_ARG, "mlp_samples: null samples");
    if (reinterpret_cast<uintptr_t>(samples) % 16)
        return ctx->fail(SPH_E_ARG, "mlp_samples: samples not 16-byte aligned");
    SPH_TRY(check_common(ctx, nb, p, params, SPH_F64, (const void* const*)u, (const void* const*)rhs,
                         "mlp_samples"));
    if (target)
        for (int c = 0; c < 3; ++c)
            if (!target[c]) return ctx->fail(SPH_E_ARG, "mlp_samples: null target vector");
    WarmOp<double> w;
    Sell<double> sell{};
    double* ucell = nullptr;
    double* info = nullptr;
    SPH_TRY(prepare<double>(ctx, nb, p, params, (const void* const*)u, &w, &sell, &ucell, &info));
    SPH_TRY((warm_samples<double, double>(ctx, w, (const void* const*)rhs, ucell, target, 1, samples, info,
                                          nullptr)));
    double Uh = 0.0;
    SPH_HIP(hipMemcpyAsync(&Uh, info + kWiU, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    SPH_HIP(hipStreamSynchronize(ctx->stream));
    if (U) *U = Uh;
    return SPH_OK;
}

extern "C" sph_status sph_mlp_warmstart(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p,
                                        const sph_visc_params* params, int32_t prec, const void* const u[3],
                                        const void* const rhs[3], const float* mlp_params, void* const x0[3],
                                        double* U) {
    if (!ctx) return SPH_E_ARG;
    if (!mlp_params || !x0) return ctx->fail(SPH_E_ARG, "mlp_warmstart: null argument");
    SPH_TRY(check_common(ctx, nb, p, params, prec, u, rhs, "mlp_warmstart"));
    for (int c = 0; c < 3; ++c)
        if (!x0[c]) return ctx->fail(SPH_E_ARG, "mlp_warmstart: null output vector");
    if (prec == SPH_F64) return warmstart_entry<double>(ctx, nb, p, params, u, rhs, mlp_params, x0, U);
    return warmstart_entry<float>(ctx, nb, p, params, u, rhs, mlp_params, x0, U);
}
