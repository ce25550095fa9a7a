// Papanastasiou viscosity from the velocity field (Section "Non-Newtonian
// viscosity", eq. papa): per particle the velocity gradient over its
// neighbours, the symmetric shear rate, its second invariant D, and
// mu = tau0 Ybar(D) + mu0 with the regularised yield term Ybar.
#include <cmath>

#include "sph_device.hpp"

namespace sph {

// Ybar(D) = (1 - exp(-m D))/D for m D >= x0, else m T(m D), T the Maclaurin
// series of (1 - e^-x)/x cut after 8 terms, in Horner form
// 1 - x/2 (1 - x/3 (... (1 - x/7 (1 - x/8)))).  The switch x0 is where the
// first omitted term x^8/9! equals single-precision epsilon (the printed
// switch "D >= m" cannot be meant: the series would then run at m D up to m^2).
__device__ inline double ybar(double D, double m, double x0) {
    const double x = m * D;
    if (x >= x0) return (1.0 - exp(-x)) / D;
    double t = 1.0;
#pragma unroll
    for (int k = 8; k >= 2; --k) t = 1.0 - x / (double)k * t;
    return m * t;
}

// One thread per particle in cell order.  G = sum_a (m_a/rho_a) F(r_ab)
// r_ab u_ab^T over the neighbours a (r_ab = r_a - r_b by minimum image,
// u_ab = u_a - u_b; the printed form, minus the usual SPH gradient, which
// the symmetric quadratic invariant does not see), S = (G + G^T)/2,
// D = sqrt(2 S:S) (the shear rate in simple shear).  Fluid rows get
// tau0 Ybar(D) + mu0, wall rows keep their viscosity; both outputs are
// written in the caller's order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_papa_visc(NbrView nv, PartView pv, const T* __restrict__ u,
                                                      const int32_t* __restrict__ perm, double tau0, double m,
                                                      double mu0, double x0, double* __restrict__ mu_out,
                                                      double* __restrict__ d_out) {
    const int64_t b = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (b >= nv.n) return;
    const Grid& g = nv.g;
    const int32_t row = (int32_t)b;
    const Pos4 pb = nv.pos[row];
    const V3<T> ub = ld3(u, row);
    double G[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for_each_neighbor(nv, row, [&](int32_t a, double r2) {
        const Pos4 pa = nv.pos[a];
        const double r[3] = {disp(pa.x, pb.x, g.period[0]), disp(pa.y, pb.y, g.period[1]),
                             disp(pa.z, pb.z, g.period[2])};
        const double F = kernel_f(g, sqrt(r2) * g.inv_h) * g.inv_h5;
        const double vf = pv.mu_mr[a].y * F;
        const V3<T> ua = ld3(u, a);
        const double du[3] = {(double)ua.x - (double)ub.x, (double)ua.y - (double)ub.y,
                              (double)ua.z - (double)ub.z};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) G[i][j] += vf * r[i] * du[j];
    });
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double s = 0.5 * (G[i][j] + G[j][i]);
            ss += s * s;
        }
    const double D = sqrt(2.0 * ss);
    const int32_t o = perm[row];
    mu_out[o] = pv.type[row] == SPH_FLUID ? tau0 * ybar(D, m, x0) + mu0 : pv.mu[row];
    if (d_out) d_out[o] = D;
}

template <typename T>
static sph_status papa_entry(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, const void* const u[3],
                             double tau0, double m, double mu0, double* mu_out, double* d_out) {
    PartView pv;
    SPH_TRY(gather_props(ctx, nb, p, &pv));
    T* ucell = nullptr;
    SPH_TRY(ctx->ensure_t(kViscU, (size_t)nb->n * 3, &ucell));
    SPH_TRY(gather_vec3<T>(ctx, nb, u, ucell));
    const double x0 = std::pow(362880.0 * std::ldexp(1.0, -23), 0.125);
    const int64_t nblk = ceil_div(nb->n, (int64_t)kBlock);
    const dim3 grid((unsigned)(nblk >= 64 ? ceil_div(nblk, (int64_t)kNumXcd) * kNumXcd : nblk));
    hipLaunchKernelGGL(k_papa_visc<T>, grid, dim3(kBlock), 0, ctx->stream, nb->view(), pv, (const T*)ucell,
                       (const int32_t*)nb->perm, tau0, m, mu0, x0, mu_out, d_out);
    SPH_LAUNCHED("k_papa_visc");
    return SPH_OK;
}

}  // namespace sph

using namespace sph;

extern "C" sph_status sph_visc_papanastasiou(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p,
                                             int32_t prec, const void* const u[3], double tau0, double m,
                                             double mu0, double* mu_out, double* shear_out) {
    if (!ctx) return SPH_E_ARG;
    if (!nb || !u || !mu_out) return ctx->fail(SPH_E_ARG, "visc_papanastasiou: null argument");
    if (nb->device != ctx->device) return ctx->fail(SPH_E_ARG, "visc_papanastasiou: handle of another device");
    for (int c = 0; c < 3; ++c)
        if (!u[c]) return ctx->fail(SPH_E_ARG, "visc_papanastasiou: null velocity component");
    if (!(tau0 >= 0.0) || !std::isfinite(tau0) || !(m > 0.0) || !std::isfinite(m) || !(mu0 >= 0.0) ||
        !std::isfinite(mu0))
        return ctx->fail(SPH_E_ARG, "visc_papanastasiou: tau0, mu0 must be finite and >= 0, m finite and > 0");
    if (prec != SPH_F64 && prec != SPH_F32) return ctx->fail(SPH_E_ARG, "visc_papanastasiou: prec");
    SPH_TRY(check_particles(ctx, nb, p));
    if (nb->n == 0) return SPH_OK;
    if (prec == SPH_F64) return papa_entry<double>(ctx, nb, p, u, tau0, m, mu0, mu_out, shear_out);
    return papa_entry<float>(ctx, nb, p, u, tau0, m, mu0, mu_out, shear_out);
}
