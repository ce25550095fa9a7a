// One step of the semi-implicit predictor/corrector (Section "Semi-implicit
// integration scheme") over the library's own calls: neighbour builds, the
// two viscous solves and the viscosity updates, with the elementwise parts
// (right-hand sides, advection) as kernels here.  The inviscid acceleration
// is the body force alone and the density stays fixed: the weakly
// compressible solver around the viscous solve is not part of this library.
#include <cmath>
#include <algorithm>
#include <cstring>

#include "sph_device.hpp"

namespace sph {

// x wrapped into [lo, lo + P) on a periodic axis (P > 0): the remainder is
// taken exactly (fmod) and shifted by P when negative.
__device__ inline double wrap_axis(double x, double lo, double P) {
    if (!(P > 0.0)) return x;
    double r = fmod(x - lo, P);
    if (r != 0.0) {
        if (r < 0.0) r += P;
    } else {
        r = 0.0;
    }
    return lo + r;
}

struct Box {
    double lo[3];
    double per[3];  // period, 0 on non-periodic axes
};

// Right-hand side of A(d) V = B: u + d g on fluid rows; the wall rows of the
// dynamic (u_w) and dummy (2 u_w) models (eqs. implicit-system-dyn-full,
// implicit-system-dummy-full), u_w being the prescribed wall velocity.
__global__ __launch_bounds__(kBlock) void k_step_rhs(int64_t n, const uint8_t* __restrict__ type,
                                                     const double* __restrict__ u0, const double* __restrict__ u1,
                                                     const double* __restrict__ u2, double g0, double g1, double g2,
                                                     double d, double wallfac, double* __restrict__ b0,
                                                     double* __restrict__ b1, double* __restrict__ b2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (type[i] == SPH_FLUID) {
        b0[i] = u0[i] + d * g0;
        b1[i] = u1[i] + d * g1;
        b2[i] = u2[i] + d * g2;
    } else {
        b0[i] = wallfac * u0[i];
        b1[i] = wallfac * u1[i];
        b2[i] = wallfac * u2[i];
    }
}

// Predictor: r* = r + (dt/2) u on fluid rows (walls stay); the wall rows of
// u* take the prescribed wall velocity (the solve leaves its internal wall
// unknowns there).
__global__ __launch_bounds__(kBlock) void k_step_half(int64_t n, const uint8_t* __restrict__ type,
                                                      const double* __restrict__ x, const double* __restrict__ y,
                                                      const double* __restrict__ z, const double* __restrict__ u0,
                                                      const double* __restrict__ u1, const double* __restrict__ u2,
                                                      double dt, Box box, double* __restrict__ px,
                                                      double* __restrict__ py, double* __restrict__ pz,
                                                      double* __restrict__ h0, double* __restrict__ h1,
                                                      double* __restrict__ h2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (type[i] == SPH_FLUID) {
        const double hd = 0.5 * dt;
        px[i] = wrap_axis(x[i] + hd * u0[i], box.lo[0], box.per[0]);
        py[i] = wrap_axis(y[i] + hd * u1[i], box.lo[1], box.per[1]);
        pz[i] = wrap_axis(z[i] + hd * u2[i], box.lo[2], box.per[2]);
    } else {
        px[i] = x[i];
        py[i] = y[i];
        pz[i] = z[i];
        h0[i] = u0[i];
        h1[i] = u1[i];
        h2[i] = u2[i];
    }
}

// Corrector: r' = r + (dt/2)(u + u') and u = u' on fluid rows; walls keep
// position and velocity.  Each thread reads its particle before writing it,
// so the outputs may alias the inputs.
__global__ __launch_bounds__(kBlock) void k_step_final(int64_t n, const uint8_t* __restrict__ type,
                                                       const double* x, const double* y, const double* z,
                                                       double* u0, double* u1, double* u2,
                                                       const double* __restrict__ v0, const double* __restrict__ v1,
                                                       const double* __restrict__ v2, double dt, Box box,
                                                       double* ox, double* oy, double* oz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i];
    if (type[i] == SPH_FLUID) {
        const double hd = 0.5 * dt;
        const double a0 = u0[i], a1 = u1[i], a2 = u2[i];
        const double n0 = v0[i], n1 = v1[i], n2 = v2[i];
        ox[i] = wrap_axis(xi + hd * (a0 + n0), box.lo[0], box.per[0]);
        oy[i] = wrap_axis(yi + hd * (a1 + n1), box.lo[1], box.per[1]);
        oz[i] = wrap_axis(zi + hd * (a2 + n2), box.lo[2], box.per[2]);
        u0[i] = n0;
        u1[i] = n1;
        u2[i] = n2;
    } else {
        ox[i] = xi;
        oy[i] = yi;
        oz[i] = zi;
    }
}

}  // namespace sph

using namespace sph;

namespace {

// Owns the neighbour handles of one step.
struct NbrGuard {
    sph_nbr* h = nullptr;
    ~NbrGuard() {
        if (h) sph_neighbors_free(h);
    }
    sph_nbr* reset(sph_nbr* x) {
        if (h) sph_neighbors_free(h);
        h = x;
        return x;
    }
};

}  // namespace

extern "C" sph_status sph_semi_implicit_step(sph_ctx* ctx, const sph_domain* dom, const sph_particles* p,
                                             const sph_visc_params* params, int32_t prec,
                                             const sph_step_params* sp, const sph_solve_opts* opts,
                                             double* const pos_out[3], double* const u[3], double* mu_out,
                                             sph_solve_report* reports) {
    if (!ctx) return SPH_E_ARG;
    if (!dom || !p || !params || !sp || !opts || !pos_out || !u || !mu_out)
        return ctx->fail(SPH_E_ARG, "semi_implicit_step: null argument");
    for (int c = 0; c < 3; ++c)
        if (!pos_out[c] || !u[c]) return ctx->fail(SPH_E_ARG, "semi_implicit_step: null array");
    if (!p->x || !p->y || !p->z || !p->mass || !p->rho || !p->mu || !p->type)
        return ctx->fail(SPH_E_ARG, "semi_implicit_step: null particle array");
    if (prec != SPH_F64 && prec != SPH_MIXED)
        return ctx->fail(SPH_E_ARG, "semi_implicit_step: prec must be SPH_F64 or SPH_MIXED (FP64 velocities)");
    if (!(params->dt >= 0.0) || !std::isfinite(params->dt)) return ctx->fail(SPH_E_ARG, "semi_implicit_step: dt");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(sp->g[c])) return ctx->fail(SPH_E_ARG, "semi_implicit_step: g must be finite");
    if (sp->papanastasiou && (!(sp->tau0 >= 0.0) || !std::isfinite(sp->tau0) || !(sp->m > 0.0) ||
                              !std::isfinite(sp->m) || !(sp->mu0 >= 0.0) || !std::isfinite(sp->mu0)))
        return ctx->fail(SPH_E_ARG, "semi_implicit_step: tau0, mu0 must be finite and >= 0, m finite and > 0");
    const int64_t n = p->n;
    if (n <= 0) return ctx->fail(SPH_E_ARG, "semi_implicit_step: no particles");
    if (n > INT32_MAX) return ctx->fail(SPH_E_OVERFLOW, "semi_implicit_step: more than 2^31 - 1 particles");
    Box box;
    for (int a = 0; a < 3; ++a) {
        box.lo[a] = dom->lo[a];
        box.per[a] = dom->periodic[a] ? dom->hi[a] - dom->lo[a] : 0.0;
    }
    const double dt = params->dt;
    const double wallfac = params->wall == SPH_WALL_DUMMY ? 2.0 : 1.0;

    // work arrays, caller order: rhs, u*, r*, mu*, u^{n+1}
    double* buf = nullptr;
    SPH_TRY(ctx->ensure_t(kStepBuf, (size_t)n * 13, &buf));
    double* rhs[3] = {buf, buf + n, buf + 2 * n};
    double* uh[3] = {buf + 3 * n, buf + 4 * n, buf + 5 * n};
    double* ph[3] = {buf + 6 * n, buf + 7 * n, buf + 8 * n};
    double* muh = buf + 9 * n;
    double* un[3] = {buf + 10 * n, buf + 11 * n, buf + 12 * n};
    const dim3 grid((unsigned)ceil_div(n, (int64_t)kBlock)), block(kBlock);

    // each solve starts from the previous velocity; a learned start
    // (opts->warm_params) takes that velocity as its u
    sph_solve_opts o = *opts;
    o.x0_given = 1;
    for (int c = 0; c < 3; ++c) o.warm_u[c] = nullptr;
    sph_solve_report rloc[2];
    sph_solve_report* rep = reports ? reports : rloc;
    if (!reports) std::memset(rloc, 0, sizeof(rloc));

    // 1. half step at r^n: A^n(dt/2) V* = u^n + (dt/2) g, from u^n
    NbrGuard nb;
    sph_nbr* h0 = nullptr;
    SPH_TRY(sph_build_neighbors(ctx, p, dom, &h0));
    nb.reset(h0);
    hipLaunchKernelGGL(k_step_rhs, grid, block, 0, ctx->stream, n, p->type, u[0], u[1], u[2], sp->g[0], sp->g[1],
                       sp->g[2], 0.5 * dt, wallfac, rhs[0], rhs[1], rhs[2]);
    SPH_LAUNCHED("k_step_rhs");
    for (int c = 0; c < 3; ++c)
        SPH_HIP(hipMemcpyAsync(uh[c], u[c], sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream));
    sph_visc_params half = *params;
    half.dt = 0.5 * dt;
    {
        const void* b[3] = {rhs[0], rhs[1], rhs[2]};
        void* x[3] = {uh[0], uh[1], uh[2]};
        const sph_status s = sph_visc_solve(ctx, nb.h, nullptr, p, &half, prec, b, x, &o, &rep[0]);
        if (s < 0) return s;
    }
    // 2. r* = r^n + (dt/2) u^n; walls of u* back to u_w; mu* = mu(r*, u*)
    hipLaunchKernelGGL(k_step_half, grid, block, 0, ctx->stream, n, p->type, p->x, p->y, p->z, u[0], u[1], u[2],
                       dt, box, ph[0], ph[1], ph[2], uh[0], uh[1], uh[2]);
    SPH_LAUNCHED("k_step_half");
    sph_particles pstar = *p;
    pstar.x = ph[0];
    pstar.y = ph[1];
    pstar.z = ph[2];
    sph_nbr* h1 = nullptr;
    SPH_TRY(sph_build_neighbors(ctx, &pstar, dom, &h1));
    nb.reset(h1);
    if (sp->papanastasiou) {
        const void* uu[3] = {uh[0], uh[1], uh[2]};
        SPH_TRY(sph_visc_papanastasiou(ctx, nb.h, &pstar, SPH_F64, uu, sp->tau0, sp->m, sp->mu0, muh, nullptr));
    } else {
        SPH_HIP(hipMemcpyAsync(muh, p->mu, sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream));
    }
    pstar.mu = muh;
    // 3. full step at r*: A*(dt) V = u^n + dt g, from u*
    hipLaunchKernelGGL(k_step_rhs, grid, block, 0, ctx->stream, n, p->type, u[0], u[1], u[2], sp->g[0], sp->g[1],
                       sp->g[2], dt, wallfac, rhs[0], rhs[1], rhs[2]);
    SPH_LAUNCHED("k_step_rhs");
    for (int c = 0; c < 3; ++c)
        SPH_HIP(hipMemcpyAsync(un[c], uh[c], sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream));
    {
        const void* b[3] = {rhs[0], rhs[1], rhs[2]};
        void* x[3] = {un[0], un[1], un[2]};
        const sph_status s = sph_visc_solve(ctx, nb.h, nullptr, &pstar, params, prec, b, x, &o, &rep[1]);
        if (s < 0) return s;
    }
    // 4. r^{n+1} = r^n + (dt/2)(u^n + u^{n+1}), u = u^{n+1} (fluid rows)
    hipLaunchKernelGGL(k_step_final, grid, block, 0, ctx->stream, n, p->type, p->x, p->y, p->z, u[0], u[1], u[2],
                       un[0], un[1], un[2], dt, box, pos_out[0], pos_out[1], pos_out[2]);
    SPH_LAUNCHED("k_step_final");
    // mu^{n+1} = mu(r^{n+1}, u^{n+1}), lagged into the next step
    if (sp->papanastasiou) {
        sph_particles pn = *p;
        pn.x = pos_out[0];
        pn.y = pos_out[1];
        pn.z = pos_out[2];
        sph_nbr* h2 = nullptr;
        SPH_TRY(sph_build_neighbors(ctx, &pn, dom, &h2));
        nb.reset(h2);
        const void* uu[3] = {u[0], u[1], u[2]};
        SPH_TRY(sph_visc_papanastasiou(ctx, nb.h, &pn, SPH_F64, uu, sp->tau0, sp->m, sp->mu0, mu_out, nullptr));
    } else if (mu_out != p->mu) {
        SPH_HIP(hipMemcpyAsync(mu_out, p->mu, sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream));
    }
    SPH_HIP(hipStreamSynchronize(ctx->stream));
    return (sph_status)std::max(rep[0].status, rep[1].status);
}
