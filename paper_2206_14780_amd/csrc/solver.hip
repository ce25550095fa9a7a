// BiCGSTAB for the three systems A V = B sharing one matrix
// (Section "Restructuring the stabilized biconjugate gradient method").
//
// One iteration is five kernels:
//   P   p = r + beta p - alpha' A p      (robust; textbook: p = r + beta (p - omega v))
//   A1  A p, and partials of delta = r0hat . A p
//   S   s = r - alpha A p                 (the paper's r_star)
//   A2  A s, and partials of s . A s, A s . A s (and s . s for the textbook check)
//   K3  x = x + alpha p + omega s, r = s - omega A s, partials of r0hat . r and r . r
// The rotated CG for symmetric systems (Section "Restructuring the Conjugate
// Gradient") takes three: P (p = r + beta p, partials of rho = <r, r>_D),
// A (A p, partials of <p, A p>_D) and K (alpha = rho / <p, A p>_D,
// x = x + alpha p, r = r - alpha A p, partials of <r, r>_D and r . r), with
// <u, v>_D = sum_i D_i u_i v_i under the Jacobi scaling (D^-1 A is
// self-adjoint in it when A is symmetric; D = 1 without scaling).
// plus, every `true_res_period` iterations, the FP64-accurate residual
// b - A x, whose outcome the next P applies (restart of a component that the
// recursion calls converged but the true residual does not).
// Every kernel that needs a scalar reduces the previous kernel's per-block
// partials itself, in a fixed order, so each block derives the same scalars
// without a host round trip or an extra launch; block 0 also records them in
// the control block.  All inner products and scalars are FP64.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "mlp.hpp"
#include "operator_kernels.hpp"

namespace sph {

constexpr int kKp = 9;  // partials per block of the close-out / initial-residual kernels

// Single-precision scalars (the paper's all-FP32 solver, appendix
// "Implementation notes"): with sc.fp32 every reduced inner product and every
// scalar of the recurrences is rounded to FP32.  The operands being FP32
// values, an operation evaluated in FP64 and rounded once equals the FP32
// operation (FP64 has more than 2 x 24 + 2 significand bits); a reduced sum
// rounded once stands for the compensated FP32 sum, which is within about a
// unit of its last place.
__device__ inline double rsc(const SolveConst& sc, double v) { return sc.fp32 ? (double)(float)v : v; }
template <int K>
__device__ inline void rsc_all(const SolveConst& sc, double (&v)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = rsc(sc, v[k]);
}

// Initial residual: r = b - A x0 given in `r0` (null: x0 = 0, r = b),
// r0hat = r; partials of r0hat . r, r . r and b . b.
template <typename T, bool KH = false>
__global__ __launch_bounds__(kMaxBlock) void k_init(int64_t n, const T* __restrict__ b, const T* __restrict__ r0,
                                                    T* __restrict__ r, T* __restrict__ rh0,
                                                    double* __restrict__ part) {
    __shared__ double lds[2 * kKp * kMaxWaves];
    double acc[kKp];
    float cmp[kKp];
#pragma unroll
    for (int k = 0; k < kKp; ++k) {
        acc[k] = 0.0;
        cmp[k] = 0.f;
    }
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t rpb = ceil_div(n, (int64_t)gridDim.x);
    const int64_t i0 = bid * rpb, i1 = min(i0 + rpb, n);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const V3<T> bv = ld3(b, i);
        const V3<T> rv = r0 ? ld3(r0, i) : bv;
        st3(r, i, rv);
        st3(rh0, i, rv);
        const double q[3] = {(double)rv.x, (double)rv.y, (double)rv.z};
        const double bb[3] = {(double)bv.x, (double)bv.y, (double)bv.z};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dot_add<KH>(acc[c], cmp[c], q[c], q[c]);
            dot_add<KH>(acc[3 + c], cmp[3 + c], q[c], q[c]);
            dot_add<KH>(acc[6 + c], cmp[6 + c], bb[c], bb[c]);
        }
    }
    write_partials_kh<kKp, KH>(acc, cmp, lds, part);
}

// Scalars of the p update of iteration `it`, i.e. the outcome of iteration
// j = it - 1 (or of the initial residual when it == 1).
struct PScalars {
    double g[3], ap[3], bt[3], rr[3], tau2[3], bb[3], trr[3], rref[3];
    int32_t state[3], stall[3], stall0[3], nres[3], restart[3];
    int32_t reason;
    int32_t nonfinite;
    int32_t checked;
};

__device__ inline void p_scalars(const Ctl* __restrict__ ctl, int32_t it, const SolveConst& sc,
                                 const double (&red)[kKp], const double (&tr)[3], bool check, PScalars& o) {
    const int32_t j = it - 1;
    const int prev = j & 1;
    o.nonfinite = 0;
    o.checked = check ? 1 : 0;
    int any_prog = 0;
    for (int c = 0; c < 3; ++c) {
        const double g = red[c];
        const double rr = red[3 + c];
        double tau2, bb;
        int stall = 0, st0 = 0;
        double ap = 0.0, bt = 0.0;
        if (it == 1) {
            bb = red[6 + c];
            tau2 = rsc(sc, sc.tol2 * bb);
            if (tau2 < sc.floor_) tau2 = sc.floor_;
            if (!finite_d(bb)) o.nonfinite = 1;
        } else {
            bb = ctl->bb[c];
            tau2 = ctl->tau2[c];
            stall = ctl->stallB[prev][c];
            if (sc.variant == SPH_ROBUST) {
                // alpha'_j = gamma_{j+1}/delta_j, beta_j = alpha'_j/omega_j
                if (!stall) {
                    ap = rsc(sc, g / ctl->delta[prev][c]);
                    if (!finite_d(ap)) ap = 0.0;
                    bt = rsc(sc, ap / ctl->omega[prev][c]);
                    if (!finite_d(bt)) bt = 0.0;
                }
                if (g == 0.0) stall = 1;
            } else if (sc.variant == SPH_CG) {
                // beta_{j+1} = rho_{j+1}/rho_j: g = <r, r>_D from the
                // close-out's partials, rho_j as the close-out stored it;
                // 0 after a stalled iteration
                if (!stall) {
                    const double rp = ctl->gam[prev][c];
                    if (rp != 0.0) bt = rsc(sc, g / rp);
                    if (!finite_d(bt)) bt = 0.0;
                }
            } else {
                // beta_{j+1} = (gamma_{j+1}/gamma_j)(alpha_j/omega_j)
                const double gp = ctl->gam[prev][c], al = ctl->alpha[prev][c], om = ctl->omega[prev][c];
                if (gp != 0.0 && om != 0.0) bt = rsc(sc, rsc(sc, g / gp) * rsc(sc, al / om));
                if (!finite_d(bt)) bt = 0.0;
            }
        }
        int32_t nres = it == 1 ? 0 : ctl->nres[prev][c];
        double rref = it == 1 ? rr : ctl->rr_ref[prev][c];
        o.restart[c] = 0;
        if (it > 1 && ctl->restart_iter == j && ctl->restart[c]) {
            // restarted by a host-issued check: fresh direction from r_true
            o.g[c] = ctl->gam_restart[c];
            o.rr[c] = ctl->rr_restart[c];
            rref = ctl->rr_restart[c];
            o.ap[c] = 0.0;
            o.bt[c] = 0.0;
            o.state[c] = o.rr[c] < tau2 ? SPH_CONVERGED : SPH_PROGRESSING;
        } else {
            o.g[c] = g;
            o.rr[c] = rr;
            o.ap[c] = ap;
            o.bt[c] = bt;
            o.state[c] = rr < tau2 ? SPH_CONVERGED : (stall ? SPH_STATE_STALLED : SPH_PROGRESSING);
        }
        if (check) {
            bool rs = false;
            if (o.state[c] == SPH_CONVERGED && !(tr[c] < tau2)) {
                // the recursion says converged, the true residual does not
                if (nres < kMaxRestarts) {
                    ++nres;
                    rs = true;
                } else {
                    o.state[c] = SPH_STATE_STALLED;
                }
            } else if (o.state[c] == SPH_PROGRESSING && tr[c] < sc.drop * rref) {
                rs = true;  // the residual has fallen far below the shadow vector
            }
            if (rs) {
                // restart from the true residual (copied by the kernel body)
                o.restart[c] = 1;
                o.g[c] = tr[c];
                o.rr[c] = tr[c];
                o.ap[c] = 0.0;
                o.bt[c] = 0.0;
                o.state[c] = tr[c] < tau2 ? SPH_CONVERGED : SPH_PROGRESSING;
                rref = tr[c];
            }
        }
        if (sc.variant == SPH_STANDARD && o.g[c] == 0.0) st0 = 1;  // breakdown of iteration it
        o.trr[c] = tr[c];
        o.nres[c] = nres;
        o.rref[c] = rref;
        o.stall[c] = stall;
        o.stall0[c] = st0;
        o.tau2[c] = tau2;
        o.bb[c] = bb;
        any_prog |= (o.state[c] == SPH_PROGRESSING);
    }
    int32_t reason = 0;
    if (!any_prog || o.nonfinite) reason |= kHaltNoProg;
    if (j >= sc.max_iter) reason |= kHaltMaxIter;
    o.reason = reason;
}

// CG: dw (null: 1) weighs the partials of rho = <r, r>_D written to
// part_rho, taken after any restart copy (the r that p is built from).
template <typename T, bool KH = false>
__global__ __launch_bounds__(kMaxBlock) void k_pupd(Ctl* __restrict__ ctl, int32_t it, SolveConst sc,
                                                    const double* __restrict__ part, int32_t nblk,
                                                    const double* __restrict__ part_tr, int64_t n, T* __restrict__ r,
                                                    T* __restrict__ rh0, T* __restrict__ p,
                                                    const T* __restrict__ ap, const T* __restrict__ rt,
                                                    double* __restrict__ hist, int32_t* __restrict__ stallhist,
                                                    const double* __restrict__ dw, double* __restrict__ part_rho) {
    if (ctl->halt) return;
    __shared__ double lds[2 * kKp * kMaxWaves];
    double red[kKp];
    reduce_partials_kh<kKp, KH>(part, nblk, red, lds);
    rsc_all(sc, red);
    const int32_t j = it - 1;
    // periodic FP64 true residual of iteration j, unless a host-issued check
    // already covered it
    const bool check = sc.true_res_period > 0 && j > 0 && j % sc.true_res_period == 0 &&
                       ctl->host_checked_iter != j;
    double tr[3] = {0.0, 0.0, 0.0};
    if (check) {
        reduce_partials<3>(part_tr, sc.tr_blocks, tr, lds);
        rsc_all(sc, tr);
    }
    PScalars s;
    p_scalars(ctl, it, sc, red, tr, check, s);
    const int cur = it & 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            ctl->gam[cur][c] = s.g[c];
            ctl->alphap[cur][c] = s.ap[c];
            ctl->beta[cur][c] = s.bt[c];
            ctl->stall0[cur][c] = s.stall0[c];
            ctl->nres[cur][c] = s.nres[c];
            ctl->rr_ref[cur][c] = s.rref[c];
            ctl->rr[c] = s.rr[c];
            ctl->state[c] = s.state[c];
            if (it == 1) {
                ctl->tau2[c] = s.tau2[c];
                ctl->bb[c] = s.bb[c];
            }
            if (j < sc.hist_cap) {
                hist[3 * j + c] = s.rr[c];
                stallhist[3 * j + c] = s.stall[c];
            }
            if (s.checked) {
                ctl->trr[c] = s.trr[c];
                ctl->n_replaced += s.restart[c];
            }
        }
        if (s.checked) {
            ctl->n_true_checks += 1;
            ctl->dev_checked_iter = j;
        }
        if (s.nonfinite) ctl->nonfinite = 1;
        ctl->halt_reason = s.reason;
        ctl->iter = s.reason ? j : it;
        if (s.reason) ctl->halt = 1;
    }
    if (s.reason) return;
    // body: p update; a zero coefficient skips its vector (the robust form
    // also serves the CG, whose alpha' is 0)
    const bool textbook = sc.variant == SPH_STANDARD;
    const bool use_p = s.bt[0] != 0.0 || s.bt[1] != 0.0 || s.bt[2] != 0.0;
    const bool use_ap = !textbook ? (s.ap[0] != 0.0 || s.ap[1] != 0.0 || s.ap[2] != 0.0) : use_p;
    const bool any_rs = s.restart[0] | s.restart[1] | s.restart[2];
    double om[3];
    for (int c = 0; c < 3; ++c) om[c] = !textbook ? 0.0 : (it > 1 ? ctl->omega[j & 1][c] : 1.0);
    double acc[3] = {0.0, 0.0, 0.0};
    float cmp[3] = {0.f, 0.f, 0.f};
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t rpb = ceil_div(n, (int64_t)gridDim.x);
    const int64_t i0 = bid * rpb, i1 = min(i0 + rpb, n);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        V3<T> rv = ld3(r, i);
        if (any_rs) {
            const V3<T> tv = ld3(rt, i);
            V3<T> hv = ld3(rh0, i);
            if (s.restart[0]) rv.x = hv.x = tv.x;
            if (s.restart[1]) rv.y = hv.y = tv.y;
            if (s.restart[2]) rv.z = hv.z = tv.z;
            st3(r, i, rv);
            st3(rh0, i, hv);
        }
        V3<T> pv{}, av{};
        if (use_p) pv = ld3(p, i);
        if (use_ap) av = ld3(ap, i);
        T o[3] = {rv.x, rv.y, rv.z};
        const T pp[3] = {pv.x, pv.y, pv.z};
        const T aa[3] = {av.x, av.y, av.z};
        for (int c = 0; c < 3; ++c) {
            if (!textbook) {
                if (s.bt[c] != 0.0) o[c] = o[c] + (T)s.bt[c] * pp[c];
                if (s.ap[c] != 0.0) o[c] = o[c] - (T)s.ap[c] * aa[c];
            } else if (s.bt[c] != 0.0) {
                o[c] = o[c] + (T)s.bt[c] * (pp[c] - (T)om[c] * aa[c]);
            }
        }
        st3(p, i, V3<T>{o[0], o[1], o[2]});
        if (part_rho) {
            const double d = dw ? dw[i] : 1.0;
            dot_add_w<KH>(acc[0], cmp[0], d, (double)rv.x, (double)rv.x);
            dot_add_w<KH>(acc[1], cmp[1], d, (double)rv.y, (double)rv.y);
            dot_add_w<KH>(acc[2], cmp[2], d, (double)rv.z, (double)rv.z);
        }
    }
    if (part_rho) write_partials_kh<3, KH>(acc, cmp, lds, part_rho);
}

// alpha_i = gamma_i/delta_i, then s = r - alpha A p.
template <typename T, bool KH = false>
__global__ __launch_bounds__(kMaxBlock) void k_supd(Ctl* __restrict__ ctl, int32_t it, SolveConst sc,
                                                    const double* __restrict__ part, int32_t nblk, int64_t n,
                                                    const T* __restrict__ r, const T* __restrict__ ap,
                                                    T* __restrict__ s) {
    if (ctl->halt) return;
    __shared__ double lds[2 * 3 * kMaxWaves];
    double red[3];
    reduce_partials_kh<3, KH>(part, nblk, red, lds);
    rsc_all(sc, red);
    const int cur = it & 1;
    double al[3];
    int32_t stall[3];
    for (int c = 0; c < 3; ++c) {
        double d = red[c];
        if (it == sc.force_stall_iter && c == sc.force_stall_comp) d = 0.0;
        red[c] = d;
        stall[c] = ctl->stall0[cur][c];
        double a = 0.0;
        if (d != 0.0 && finite_d(d)) a = rsc(sc, ctl->gam[cur][c] / d);
        if (!finite_d(a) || d == 0.0 || !finite_d(d)) {
            a = 0.0;
            stall[c] = 1;
        }
        al[c] = a;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            ctl->delta[cur][c] = red[c];
            ctl->alpha[cur][c] = al[c];
            ctl->stallA[cur][c] = stall[c];
        }
    }
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t rpb = ceil_div(n, (int64_t)gridDim.x);
    const int64_t i0 = bid * rpb, i1 = min(i0 + rpb, n);
    const T a0 = (T)al[0], a1 = (T)al[1], a2 = (T)al[2];
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const V3<T> rv = ld3(r, i);
        const V3<T> av = ld3(ap, i);
        st3(s, i, V3<T>{rv.x - a0 * av.x, rv.y - a1 * av.y, rv.z - a2 * av.z});
    }
}

// omega_i = (s . A s)/(A s . A s); x = x + alpha p + omega s; r = s - omega A s;
// partials of r0hat . r and r . r.  x is held in X (T, or FP64 under an FP32
// operator: then the update is evaluated in FP64).
template <typename T, int KA, typename X, bool KH = false>
__global__ __launch_bounds__(kMaxBlock) void k_close(Ctl* __restrict__ ctl, int32_t it, SolveConst sc,
                                                     const double* __restrict__ part, int32_t nblk, int64_t n,
                                                     X* __restrict__ x, const T* __restrict__ p,
                                                     const T* __restrict__ s, const T* __restrict__ as,
                                                     T* __restrict__ r, const T* __restrict__ rh0,
                                                     double* __restrict__ part_out) {
    if (ctl->halt) return;
    __shared__ double lds[2 * kKp * kMaxWaves];
    double red[KA];
    reduce_partials_kh<KA, KH>(part, nblk, red, lds);
    rsc_all(sc, red);
    const int cur = it & 1;
    double om[3], al[3];
    int32_t stall[3];
    for (int c = 0; c < 3; ++c) {
        const double ts = red[c], tt = red[3 + c];
        double w = 0.0;
        if (tt != 0.0) w = rsc(sc, ts / tt);
        if (!finite_d(w)) w = 0.0;
        stall[c] = ctl->stallA[cur][c] | (w == 0.0 ? 1 : 0);
        if constexpr (KA == 9) {
            if (red[6 + c] < ctl->tau2[c]) w = 0.0;  // r_star already meets the threshold
        }
        om[c] = w;
        al[c] = ctl->alpha[cur][c];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            ctl->omega[cur][c] = om[c];
            ctl->stallB[cur][c] = stall[c];
        }
    }
    double acc[kKp];
    float cmp[kKp];
#pragma unroll
    for (int k = 0; k < kKp; ++k) {
        acc[k] = 0.0;
        cmp[k] = 0.f;
    }
    const T A[3] = {(T)al[0], (T)al[1], (T)al[2]};
    const T W[3] = {(T)om[0], (T)om[1], (T)om[2]};
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t rpb = ceil_div(n, (int64_t)gridDim.x);
    const int64_t i0 = bid * rpb, i1 = min(i0 + rpb, n);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const V3<X> xv = ld3(x, i);
        const V3<T> pv = ld3(p, i), sv = ld3(s, i), av = ld3(as, i), hv = ld3(rh0, i);
        const X xx[3] = {xv.x, xv.y, xv.z};
        const T pp[3] = {pv.x, pv.y, pv.z}, ss[3] = {sv.x, sv.y, sv.z};
        const T aa[3] = {av.x, av.y, av.z}, hh[3] = {hv.x, hv.y, hv.z};
        X xo[3];
        T ro[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (sizeof(X) == sizeof(T)) {
                const T t = xx[c] + A[c] * pp[c];
                xo[c] = t + W[c] * ss[c];
            } else {
                const double t = (double)xx[c] + al[c] * (double)pp[c];
                xo[c] = t + om[c] * (double)ss[c];
            }
            ro[c] = ss[c] - W[c] * aa[c];
            dot_add<KH>(acc[c], cmp[c], (double)hh[c], (double)ro[c]);
            dot_add<KH>(acc[3 + c], cmp[3 + c], (double)ro[c], (double)ro[c]);
        }
        st3(x, i, V3<X>{xo[0], xo[1], xo[2]});
        st3(r, i, V3<T>{ro[0], ro[1], ro[2]});
    }
    write_partials_kh<kKp, KH>(acc, cmp, lds, part_out);
}

// CG close-out: alpha = rho / <p, A p>_D (0, and the component stalled,
// when that is zero or not finite); x = x + alpha p; r = r - alpha A p;
// partials (kKp per block) of <r, r>_D, r . r and three zeros, the layout
// the p update reads.  rho_i is stored as gam[it & 1] for the next beta.
template <typename T, typename X, bool KH = false>
__global__ __launch_bounds__(kMaxBlock) void k_cg_close(Ctl* __restrict__ ctl, int32_t it, SolveConst sc,
                                                        const double* __restrict__ part_rho, int32_t nrho,
                                                        const double* __restrict__ part_pap, int32_t npap,
                                                        int64_t n, X* __restrict__ x, const T* __restrict__ p,
                                                        const T* __restrict__ ap, T* __restrict__ r,
                                                        const double* __restrict__ dw,
                                                        double* __restrict__ part_out) {
    if (ctl->halt) return;
    __shared__ double lds[2 * kKp * kMaxWaves];
    double rho[3], pap[3];
    reduce_partials_kh<3, KH>(part_rho, nrho, rho, lds);
    reduce_partials_kh<3, KH>(part_pap, npap, pap, lds);
    rsc_all(sc, rho);
    rsc_all(sc, pap);
    const int cur = it & 1;
    double al[3];
    int32_t stall[3];
    for (int c = 0; c < 3; ++c) {
        double d = pap[c];
        if (it == sc.force_stall_iter && c == sc.force_stall_comp) d = 0.0;
        pap[c] = d;
        double a = 0.0;
        if (d != 0.0 && finite_d(d)) a = rsc(sc, rho[c] / d);
        stall[c] = 0;
        if (!finite_d(a) || a == 0.0) {
            a = 0.0;
            stall[c] = 1;
        }
        al[c] = a;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            ctl->gam[cur][c] = rho[c];
            ctl->delta[cur][c] = pap[c];
            ctl->alpha[cur][c] = al[c];
            ctl->stallB[cur][c] = stall[c];
        }
    }
    double acc[kKp];
    float cmp[kKp];
#pragma unroll
    for (int k = 0; k < kKp; ++k) {
        acc[k] = 0.0;
        cmp[k] = 0.f;
    }
    const T A[3] = {(T)al[0], (T)al[1], (T)al[2]};
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t rpb = ceil_div(n, (int64_t)gridDim.x);
    const int64_t i0 = bid * rpb, i1 = min(i0 + rpb, n);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const V3<X> xv = ld3(x, i);
        const V3<T> pv = ld3(p, i), av = ld3(ap, i), rv = ld3(r, i);
        const X xx[3] = {xv.x, xv.y, xv.z};
        const T pp[3] = {pv.x, pv.y, pv.z}, aa[3] = {av.x, av.y, av.z}, rr[3] = {rv.x, rv.y, rv.z};
        const double d = dw ? dw[i] : 1.0;
        X xo[3];
        T ro[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (sizeof(X) == sizeof(T)) xo[c] = xx[c] + A[c] * pp[c];
            else xo[c] = (double)xx[c] + al[c] * (double)pp[c];
            ro[c] = rr[c] - A[c] * aa[c];
            dot_add_w<KH>(acc[c], cmp[c], d, (double)ro[c], (double)ro[c]);
            dot_add<KH>(acc[3 + c], cmp[3 + c], (double)ro[c], (double)ro[c]);
        }
        st3(x, i, V3<X>{xo[0], xo[1], xo[2]});
        st3(r, i, V3<T>{ro[0], ro[1], ro[2]});
    }
    write_partials_kh<kKp, KH>(acc, cmp, lds, part_out);
}

// CG start: wall rows (identity rows of the dynamic-wall system) take their
// exact value, so r and p stay zero there and the iteration runs on the
// symmetric fluid block (Section "Linear system properties and resolution").
template <typename X>
__global__ __launch_bounds__(kBlock) void k_cg_walls(int64_t n, const uint8_t* __restrict__ type,
                                                     const double* __restrict__ b64, X* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || type[i] == SPH_FLUID) return;
    const V3<double> b = ld3(b64, i);
    st3(x, i, V3<X>{(X)b.x, (X)b.y, (X)b.z});
}

// Host-issued residual check, step 2 (one block): decide which converged
// components failed the FP64 true residual and must restart.
__global__ __launch_bounds__(kMaxBlock) void k_check_decide(Ctl* __restrict__ ctl, const double* __restrict__ part,
                                                            int32_t nblk, SolveConst sc) {
    __shared__ double lds[3 * kMaxWaves];
    double red[3];
    reduce_partials<3>(part, nblk, red, lds);
    rsc_all(sc, red);
    if (threadIdx.x != 0) return;
    const int32_t j = ctl->iter;
    ctl->n_true_checks += 1;
    for (int c = 0; c < 3; ++c) {
        ctl->trr[c] = red[c];
        int rs = 0;
        if (ctl->state[c] == SPH_CONVERGED && !(red[c] < ctl->tau2[c])) {
            if (ctl->nres[j & 1][c] < kMaxRestarts) {
                rs = 1;
                ctl->state[c] = SPH_PROGRESSING;
                ctl->nres[j & 1][c] += 1;
                ctl->n_replaced += 1;
            } else {
                ctl->state[c] = SPH_STATE_STALLED;
            }
        }
        ctl->restart[c] = rs;
    }
    ctl->restart_iter = j;
    ctl->host_checked_iter = j;
}

// Step 3: r = r0hat = r_true for restarted components, and partials of the
// new r0hat . r, r . r.
template <typename T, bool KH = false>
__global__ __launch_bounds__(kMaxBlock) void k_check_copy(const Ctl* __restrict__ ctl, int64_t n,
                                                          const T* __restrict__ rt, T* __restrict__ r,
                                                          T* __restrict__ rh0, double* __restrict__ part) {
    __shared__ double lds[2 * 6 * kMaxWaves];
    double acc[6];
    float cmp[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        acc[k] = 0.0;
        cmp[k] = 0.f;
    }
    const int rs[3] = {ctl->restart[0], ctl->restart[1], ctl->restart[2]};
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t rpb = ceil_div(n, (int64_t)gridDim.x);
    const int64_t i0 = bid * rpb, i1 = min(i0 + rpb, n);
    if (rs[0] | rs[1] | rs[2]) {
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
            const V3<T> tv = ld3(rt, i);
            V3<T> rv = ld3(r, i), hv = ld3(rh0, i);
            if (rs[0]) rv.x = hv.x = tv.x;
            if (rs[1]) rv.y = hv.y = tv.y;
            if (rs[2]) rv.z = hv.z = tv.z;
            st3(r, i, rv);
            st3(rh0, i, hv);
            const double q[3] = {(double)rv.x, (double)rv.y, (double)rv.z};
            for (int c = 0; c < 3; ++c) {
                dot_add<KH>(acc[c], cmp[c], q[c], q[c]);
                dot_add<KH>(acc[3 + c], cmp[3 + c], q[c], q[c]);
            }
        }
    }
    write_partials_kh<6, KH>(acc, cmp, lds, part);
}

template <bool KH = false>
__global__ __launch_bounds__(kMaxBlock) void k_check_finish(Ctl* __restrict__ ctl, const double* __restrict__ part,
                                                            int32_t nblk, SolveConst sc) {
    __shared__ double lds[2 * 6 * kMaxWaves];
    double red[6];
    reduce_partials_kh<6, KH>(part, nblk, red, lds);
    rsc_all(sc, red);
    if (threadIdx.x != 0) return;
    for (int c = 0; c < 3; ++c) {
        ctl->gam_restart[c] = red[c];
        ctl->rr_restart[c] = red[3 + c];
    }
}

// Final FP64 true residual, reduced into ctl->trr (one block).
__global__ __launch_bounds__(kMaxBlock) void k_final_trr(Ctl* __restrict__ ctl, const double* __restrict__ part,
                                                         int32_t nblk) {
    __shared__ double lds[3 * kMaxWaves];
    double red[3];
    reduce_partials<3>(part, nblk, red, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) ctl->trr[c] = red[c];
}

__global__ void k_ctl_init(Ctl* ctl) {
    int32_t* w = reinterpret_cast<int32_t*>(ctl);
    for (size_t i = threadIdx.x; i < sizeof(Ctl) / sizeof(int32_t); i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl->host_checked_iter = -1;
        ctl->dev_checked_iter = -1;
        ctl->restart_iter = -1;
    }
}

// rhs in caller order (precision C) -> b64 = D^-1 B in FP64 and b = rounded
// copy, cell order.
template <typename T, typename C>
__global__ __launch_bounds__(kBlock) void k_prep_rhs(int64_t n, const int32_t* __restrict__ perm,
                                                     const C* __restrict__ b0, const C* __restrict__ b1,
                                                     const C* __restrict__ b2, const double* __restrict__ diag64,
                                                     int32_t jacobi, double* __restrict__ b64,
                                                     T* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t o = perm[i];
    double v[3] = {(double)b0[o], (double)b1[o], (double)b2[o]};
    if (jacobi) {
        const double d = diag64[i];
        for (int c = 0; c < 3; ++c) v[c] = v[c] / d;
    }
    st3(b64, i, V3<double>{v[0], v[1], v[2]});
    st3(b, i, V3<T>{(T)v[0], (T)v[1], (T)v[2]});
}

}  // namespace sph

using namespace sph;

namespace {

sph_status read_ctl(sph_ctx* ctx, const Ctl* d, Ctl* h) {
    SPH_HIP(hipMemcpyAsync(h, d, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
    SPH_HIP(hipStreamSynchronize(ctx->stream));
    return SPH_OK;
}

// T: precision of the operator and of the Krylov vectors; X: precision of
// the solution and of the caller's arrays (X = T, or FP64 under an FP32
// operator).  KH: the paper's single-precision arithmetic (T = X = float):
// compensated FP32 inner products and gemv over the FP32 matrix of
// cell-relative positions (the true residual stays FP64).
template <typename T, typename X, bool KH = false>
struct Solver {
    sph_ctx* ctx;
    const sph_nbr* nb;
    PartView pv;
    OpParams op;
    int32_t mode;
    Sell<T> sell{};
    const double* diag64 = nullptr;
    const double* dw = nullptr;  // CG inner-product weights: D under the Jacobi scaling, else null (1)
    Launch L;
    T *b, *r, *rh0, *p, *ap, *s, *as, *tmp;
    X* x;
    double* b64;
    double *pa1, *pa2, *pk3, *ptr, *pchk;
    Ctl* ctl;
    double* hist;
    int32_t* stallhist;
    SolveConst sc;
    int32_t launches = 0;
    int32_t issued_iters = 0;  // iterations queued over all rounds
    // profiling of the A r_star launches: (iteration, issue round, event pair)
    int32_t profile = 0;  // time the A r_star launch of every profile-th iteration
    int32_t round = 0;
    struct Rec {
        int32_t it, round, ev;
    };
    std::vector<Rec> recs;
    std::vector<int32_t> round_end;  // last executed iteration of each round

    sph_status prof_event(int idx, hipEvent_t* out) {
        while ((int)ctx->prof_ev.size() <= idx) {
            hipEvent_t e;
            SPH_HIP(hipEventCreate(&e));
            ctx->prof_ev.push_back(e);
        }
        *out = ctx->prof_ev[idx];
        return SPH_OK;
    }

    dim3 ga() const { return dim3(L.grid_apply); }
    dim3 ba() const { return dim3(L.block_apply); }
    dim3 gs() const { return dim3(L.grid_stream); }
    dim3 bs() const { return dim3(L.block_stream); }

    // y = A x fused with the dot products of mode MODE (x of precision XT:
    // T, or X for the true residual); kDotCG weighs its products by dw
    template <int MODE, typename XT = T>
    void apply(const int32_t* halt, const XT* xin, T* yout, const T* w, double* part) {
        const double* aux = MODE == kDotCG ? dw : b64;
        if (mode == SPH_OP_CACHED)
            hipLaunchKernelGGL((k_apply_sell<T, MODE, XT, KH && MODE != kDotResid>), ga(), ba(), 0, ctx->stream,
                               halt, L.n, sell, xin, yout, w, aux, part);
        else
            hipLaunchKernelGGL((k_apply_otf<T, MODE, XT>), ga(), ba(), 0, ctx->stream, halt, nb->view(), pv, op,
                               xin, yout, w, aux, part);
        ++launches;
    }

    // events around the timed operator launch of iteration `it`
    sph_status time_begin(int32_t it, hipEvent_t* ev1) {
        *ev1 = nullptr;
        if (!(profile > 0 && it % profile == 0)) return SPH_OK;
        const int k = (int)recs.size();
        hipEvent_t ev0 = nullptr;
        SPH_TRY(prof_event(2 * k, &ev0));
        SPH_TRY(prof_event(2 * k + 1, ev1));
        recs.push_back(Rec{it, round, k});
        SPH_HIP(hipEventRecord(ev0, ctx->stream));
        return SPH_OK;
    }

    // rotated CG: P (p and the partials of rho), A (A p, <p, A p>_D), K
    sph_status iteration_cg(int32_t it) {
        const int32_t* halt = &ctl->halt;
        hipLaunchKernelGGL((k_pupd<T, KH>), gs(), bs(), 0, ctx->stream, ctl, it, sc, pk3, L.grid_stream,
                           (const double*)ptr, L.n, r, rh0, p, ap, tmp, hist, stallhist, dw, pa2);
        hipEvent_t ev1 = nullptr;
        SPH_TRY(time_begin(it, &ev1));
        apply<kDotCG>(halt, p, ap, nullptr, pa1);
        if (ev1) SPH_HIP(hipEventRecord(ev1, ctx->stream));
        hipLaunchKernelGGL((k_cg_close<T, X, KH>), gs(), bs(), 0, ctx->stream, ctl, it, sc, (const double*)pa2,
                           L.grid_stream, (const double*)pa1, L.grid_apply, L.n, x, p, ap, r, dw, pk3);
        launches += 2;
        if (sc.true_res_period > 0 && it % sc.true_res_period == 0) true_residual(halt, ptr);
        return SPH_OK;
    }

    sph_status iteration(int32_t it) {
        if (sc.variant == SPH_CG) return iteration_cg(it);
        const int32_t* halt = &ctl->halt;
        hipLaunchKernelGGL((k_pupd<T, KH>), gs(), bs(), 0, ctx->stream, ctl, it, sc, pk3, L.grid_stream,
                           (const double*)ptr, L.n, r, rh0, p, ap, tmp, hist, stallhist, (const double*)nullptr,
                           (double*)nullptr);
        apply<kDotA1>(halt, p, ap, rh0, pa1);
        hipLaunchKernelGGL((k_supd<T, KH>), gs(), bs(), 0, ctx->stream, ctl, it, sc, pa1, L.grid_apply, L.n, r, ap,
                           s);
        hipEvent_t ev1 = nullptr;
        SPH_TRY(time_begin(it, &ev1));
        const bool timed = ev1 != nullptr;
        if (sc.variant == SPH_STANDARD) {
            apply<kDotA2Std>(halt, s, as, nullptr, pa2);
            if (timed) SPH_HIP(hipEventRecord(ev1, ctx->stream));
            hipLaunchKernelGGL((k_close<T, 9, X, KH>), gs(), bs(), 0, ctx->stream, ctl, it, sc, pa2, L.grid_apply,
                               L.n, x, p, s, as, r, rh0, pk3);
        } else {
            apply<kDotA2>(halt, s, as, nullptr, pa2);
            if (timed) SPH_HIP(hipEventRecord(ev1, ctx->stream));
            hipLaunchKernelGGL((k_close<T, 6, X, KH>), gs(), bs(), 0, ctx->stream, ctl, it, sc, pa2, L.grid_apply,
                               L.n, x, p, s, as, r, rh0, pk3);
        }
        launches += 3;
        // the next p update applies the periodic FP64 residual check
        if (sc.true_res_period > 0 && it % sc.true_res_period == 0) true_residual(halt, ptr);
        return SPH_OK;
    }

    // FP64-accurate b - A x of the current x into tmp, partials into `part`.
    void true_residual(const int32_t* halt, double* part) { apply<kDotResid, X>(halt, x, tmp, nullptr, part); }

    void host_check() {
        true_residual(nullptr, pchk);
        hipLaunchKernelGGL(k_check_decide, dim3(1), dim3(kMaxBlock), 0, ctx->stream, ctl, pchk, L.grid_apply, sc);
        hipLaunchKernelGGL((k_check_copy<T, KH>), gs(), bs(), 0, ctx->stream, ctl, L.n, tmp, r, rh0,
                           pchk + 3 * (size_t)L.grid_apply);
        hipLaunchKernelGGL(k_check_finish<KH>, dim3(1), dim3(kMaxBlock), 0, ctx->stream, ctl,
                           pchk + 3 * (size_t)L.grid_apply, L.grid_stream, sc);
        launches += 3;
    }
};

template <typename T, typename X, bool KH = false>
sph_status solve_impl(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* part, const sph_visc_params* vp,
                      int32_t prec, const void* const rhs[3], void* const xout[3], const sph_solve_opts* o,
                      sph_solve_report* rep) {
    Solver<T, X, KH> S;
    S.ctx = ctx;
    S.nb = nb;
    // the paper's single precision keeps its FP32 matrix like the cached operator
    S.mode = vp->op_mode == SPH_OP_PAPER32 ? SPH_OP_CACHED : vp->op_mode;
    S.op = OpParams{vp->dt, vp->wall, vp->avg, vp->jacobi ? 1 : 0};
    S.op.f32cell = KH ? 1 : 0;
    const int64_t n = nb->n;
    S.L = make_launch(n);
    const Launch& L = S.L;
    hipEvent_t e0 = ctx->ev[0], e1 = ctx->ev[1], e2 = ctx->ev[2];
    SPH_HIP(hipEventRecord(e0, ctx->stream));

    SPH_TRY(gather_props(ctx, nb, part, &S.pv));
    ++S.launches;
    S.profile = std::max(o->profile, 0);
    if (S.mode == SPH_OP_CACHED) {
        SPH_TRY(build_sell<T>(ctx, nb, S.pv, S.op, &S.sell, &S.diag64, &rep->mat_nnz, &rep->mat_slots));
        S.launches += 6;
    } else {
        SPH_TRY(row_diag64(ctx, nb, S.pv, S.op, &S.diag64));
        ++S.launches;
    }
    const size_t v3 = (size_t)n * 3;
    SPH_TRY(ctx->ensure_t(kVecB, v3, &S.b));
    SPH_TRY(ctx->ensure_t(kVecX, v3, &S.x));  // X
    SPH_TRY(ctx->ensure_t(kVecR, v3, &S.r));
    SPH_TRY(ctx->ensure_t(kVecRh0, v3, &S.rh0));
    SPH_TRY(ctx->ensure_t(kVecP, v3, &S.p));
    SPH_TRY(ctx->ensure_t(kVecAp, v3, &S.ap));
    SPH_TRY(ctx->ensure_t(kVecS, v3, &S.s));
    SPH_TRY(ctx->ensure_t(kVecAs, v3, &S.as));
    SPH_TRY(ctx->ensure_t(kVecTmp, v3, &S.tmp));
    SPH_TRY(ctx->ensure_t(kB64, v3, &S.b64));
    SPH_TRY(ctx->ensure_t(kPartA1, (size_t)L.grid_apply * 3, &S.pa1));
    SPH_TRY(ctx->ensure_t(kPartA2, (size_t)L.grid_apply * 9, &S.pa2));
    SPH_TRY(ctx->ensure_t(kPartK3, (size_t)L.grid_stream * kKp, &S.pk3));
    // [host check: residual (3 per apply block), copy (6 per stream block) |
    //  periodic device check: residual (3 per apply block)]
    SPH_TRY(ctx->ensure_t(kPartChk, (size_t)L.grid_apply * 6 + (size_t)L.grid_stream * 6, &S.pchk));
    S.ptr = S.pchk + 3 * (size_t)L.grid_apply + 6 * (size_t)L.grid_stream;
    SPH_TRY(ctx->ensure_t(kCtl, 1, &S.ctl));
    const int32_t hist_rows = o->max_iter + 1;
    SPH_TRY(ctx->ensure_t(kHist, (size_t)hist_rows * 3, &S.hist));
    SPH_TRY(ctx->ensure_t(kStallHist, (size_t)hist_rows * 3, &S.stallhist));

    S.sc.fp32 = (o->fp32_scalars || KH) ? 1 : 0;
    if (S.sc.fp32) {
        const float tf = (float)o->tol;
        S.sc.tol2 = (double)(tf * tf);
    } else {
        S.sc.tol2 = o->tol * o->tol;
    }
    const bool vec32 = sizeof(T) == 4;
    const bool cg = o->variant == SPH_CG;
    // the drop restart renews the BiCGSTAB's shadow vector; the CG has none
    S.sc.drop = cg ? 0.0 : (o->restart_drop >= 0.0 ? o->restart_drop : 0.1);
    S.dw = cg && S.op.jacobi ? S.diag64 : nullptr;
    S.sc.tr_blocks = L.grid_apply;
    S.sc.floor_ = o->floor >= 0.0 ? o->floor : (vec32 ? (double)FLT_MIN : DBL_MIN);
    S.sc.max_iter = o->max_iter;
    S.sc.variant = o->variant;
    S.sc.true_res_period = o->true_res_period;
    S.sc.force_stall_iter = o->force_stall_iter;
    S.sc.force_stall_comp = o->force_stall_comp;
    S.sc.hist_cap = hist_rows;

    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, ctx->stream, S.ctl);
    hipLaunchKernelGGL((k_prep_rhs<T, X>), dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, ctx->stream, n,
                       nb->perm, (const X*)rhs[0], (const X*)rhs[1], (const X*)rhs[2], S.diag64, S.op.jacobi,
                       S.b64, S.b);
    S.launches += 2;
    const T* r0 = nullptr;
    double* winfo = nullptr;
    if (o->warm_params) {
        // learned start (x_l in s, its residual in as) against the plain
        // start (x, its residual in tmp), per component by true r.r
        SPH_HIP(hipEventRecord(ctx->ev[5], ctx->stream));
        SPH_TRY(ctx->ensure_t(kWarmInfo, kWiSize, &winfo));
        // u: warm_u, or per null component the initial guess (x0_given) or
        // b.  When u is the plain start itself and the matrix is cached, the
        // feature pass also yields the plain start's residual.
        const bool u_is_x0 = o->x0_given && !o->warm_u[0] && !o->warm_u[1] && !o->warm_u[2];
        const bool fuse = u_is_x0 && S.mode == SPH_OP_CACHED;
        if (o->x0_given) SPH_TRY(gather_vec3<X>(ctx, nb, (const void* const*)xout, S.x));
        const X* ucell = S.x;
        if (!u_is_x0) {
            const void* uu[3];
            for (int c = 0; c < 3; ++c) uu[c] = o->warm_u[c] ? o->warm_u[c] : (o->x0_given ? xout[c] : rhs[c]);
            X* ub = nullptr;
            SPH_TRY(ctx->ensure_t(kWarmU, v3, &ub));
            SPH_TRY(gather_vec3<X>(ctx, nb, uu, ub));
            ucell = ub;
        }
        double* pl = S.pchk;
        double* pp = S.pchk + 3 * (size_t)L.grid_apply;
        int32_t np = L.grid_apply;
        PlainResidual<T> pr{S.b64, S.tmp, nullptr};
        if (fuse) {
            SPH_TRY(ctx->ensure_t(kWarmPart2, 3 * (size_t)kWarmFeatBlocks, &pp));
            pr.part = pp;
            np = (int32_t)std::min<int64_t>(ceil_div(n, kBlock), kWarmFeatBlocks);
        }
        const WarmOp<T> w{nb, S.pv, S.op, S.mode, &S.sell, S.diag64};
        SPH_TRY((warm_learned<T, X>(ctx, w, rhs, ucell, o->warm_params, S.s, winfo, fuse ? &pr : nullptr)));
        S.template apply<kDotResid, T>(nullptr, S.s, S.as, nullptr, pl);
        if (!fuse) {
            if (o->x0_given) {
                S.template apply<kDotResid, X>(nullptr, S.x, S.tmp, nullptr, pp);
            } else {
                SPH_HIP(hipMemsetAsync(S.x, 0, sizeof(X) * v3, ctx->stream));
                SPH_TRY(warm_zero_rr(ctx, n, L.grid_apply, S.b64, pp));
            }
        }
        SPH_TRY((warm_select<T, X>(ctx, n, L.grid_stream, L.block_stream, pl, L.grid_apply, pp, np, o->x0_given,
                                   S.x, S.s, S.as, S.b, S.tmp, winfo)));
        r0 = S.tmp;
        S.launches += 11;
        SPH_HIP(hipEventRecord(ctx->ev[6], ctx->stream));
    } else if (o->x0_given) {
        SPH_TRY(gather_vec3<X>(ctx, nb, (const void* const*)xout, S.x));
    } else {
        SPH_HIP(hipMemsetAsync(S.x, 0, sizeof(X) * v3, ctx->stream));
    }
    if (cg) {
        // the CG starts the wall rows at their exact value
        hipLaunchKernelGGL(k_cg_walls<X>, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, ctx->stream, n,
                           S.pv.type, (const double*)S.b64, S.x);
        ++S.launches;
    }
    if (cg || (!o->warm_params && o->x0_given)) {
        // r0 = b - A x0 with the FP64-accurate operator
        S.true_residual(nullptr, S.pchk);
        r0 = S.tmp;
        ++S.launches;
    }
    SPH_HIP(hipMemsetAsync(S.p, 0, sizeof(T) * v3, ctx->stream));
    SPH_HIP(hipMemsetAsync(S.ap, 0, sizeof(T) * v3, ctx->stream));
    hipLaunchKernelGGL((k_init<T, KH>), S.gs(), S.bs(), 0, ctx->stream, n, S.b, r0, S.r, S.rh0, S.pk3);
    ++S.launches;
    SPH_LAUNCHED("solve setup");
    SPH_HIP(hipEventRecord(e1, ctx->stream));

    // Iterate.  The host issues iterations in batches (sized by IssuePlan)
    // and reads the device's control block one batch behind; kernels issued
    // after a halt return at once.
    CtlPoll* mail = static_cast<CtlPoll*>(ctx->host_mail);
    IssuePlan plan(o->poll_every > 0 ? o->poll_every : 8);
    const int32_t last_it = o->max_iter + 1;  // P of this iteration always halts
    int32_t j = 0;
    Ctl hctl;
    for (;;) {
        const int32_t j0 = j;
        int32_t it = j + 1;
        if (j > 0) {
            // the round starts after the residual check of iteration j: the
            // state of the pupd of j + 1, with the true residuals
            CtlPoll m;
            std::memcpy(&m, &hctl.rr, sizeof(CtlPoll));
            for (int c = 0; c < 3; ++c) m.rr[c] = hctl.trr[c];
            m.iter = j + 1;
            m.halt = 0;
            plan.restart(m);
        }
        int pend[2], npend = 0, batch = 0;
        bool halted = false;
        while (!halted) {
            const int k = it <= last_it && npend < 2 ? plan.batch(it, npend > 0) : 0;
            if (k > 0) {
                for (int q = 0; q < k && it <= last_it; ++q) SPH_TRY(S.iteration(it++));
                SPH_LAUNCHED("iteration kernels");
                const int slot = batch++ & 1;
                SPH_HIP(hipMemcpyAsync(&mail[slot], &S.ctl->rr, sizeof(CtlPoll), hipMemcpyDeviceToHost,
                                       ctx->stream));
                SPH_HIP(hipEventRecord(ctx->ev[3 + slot], ctx->stream));
                pend[npend++] = slot;
            }
            // read the older poll once two are in flight, or when nothing is
            // to be issued before it
            if (npend == 2 || (npend > 0 && k == 0)) {
                const int slot = pend[0];
                pend[0] = pend[1];
                --npend;
                SPH_HIP(hipEventSynchronize(ctx->ev[3 + slot]));
                if (mail[slot].halt) halted = true;
                else plan.observe(mail[slot]);
            } else if (it > last_it && npend == 0) {
                halted = true;
            }
        }
        S.issued_iters += (it - 1) - j0;
        SPH_TRY(read_ctl(ctx, S.ctl, &hctl));
        if (hctl.nonfinite) return ctx->fail(SPH_E_NONFINITE, "visc_solve: non-finite right-hand side");
        if (!hctl.halt) return ctx->fail(SPH_E_HIP, "visc_solve: iteration issue ended without a halt");
        j = hctl.iter;
        S.round_end.push_back(j);
        ++S.round;
        if ((hctl.halt_reason & kHaltNoProg) && hctl.dev_checked_iter != j && hctl.host_checked_iter != j) {
            S.host_check();
            SPH_LAUNCHED("residual check");
            SPH_TRY(read_ctl(ctx, S.ctl, &hctl));
        }
        bool any_prog = false;
        for (int c = 0; c < 3; ++c) any_prog |= hctl.state[c] == SPH_PROGRESSING;
        if (!any_prog || j >= o->max_iter) break;
        SPH_HIP(hipMemsetAsync(&S.ctl->halt, 0, sizeof(int32_t), ctx->stream));
    }
    // FP64 true residual of the final x for the report, unless the last check covered it
    if (hctl.dev_checked_iter != j && hctl.host_checked_iter != j) {
        S.true_residual(nullptr, S.pchk);
        hipLaunchKernelGGL(k_final_trr, dim3(1), dim3(kMaxBlock), 0, ctx->stream, S.ctl, S.pchk, L.grid_apply);
        S.launches += 1;
    }
    SPH_TRY(scatter_vec3<X>(ctx, nb, S.x, xout));
    ++S.launches;
    SPH_LAUNCHED("solve finish");
    SPH_HIP(hipEventRecord(e2, ctx->stream));
    SPH_TRY(read_ctl(ctx, S.ctl, &hctl));

    rep->iters = hctl.iter;
    int any_prog = 0, any_stall = 0;
    for (int c = 0; c < 3; ++c) {
        rep->state[c] = hctl.state[c];
        rep->rr[c] = hctl.rr[c];
        rep->bb[c] = hctl.bb[c];
        rep->tau2[c] = hctl.tau2[c];
        rep->true_rr[c] = hctl.trr[c];
        any_prog |= hctl.state[c] == SPH_PROGRESSING;
        any_stall |= hctl.state[c] == SPH_STATE_STALLED;
    }
    rep->n_true_checks = hctl.n_true_checks;
    rep->n_replaced = hctl.n_replaced;
    const int32_t rows = std::min(hctl.iter + 1, hist_rows);
    std::vector<int32_t> sh((size_t)rows * 3);
    SPH_HIP(hipMemcpyAsync(sh.data(), S.stallhist, sizeof(int32_t) * sh.size(), hipMemcpyDeviceToHost, ctx->stream));
    SPH_HIP(hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < 3; ++c) {
        int32_t cnt = 0;
        for (int32_t q = 1; q < rows; ++q) cnt += sh[(size_t)q * 3 + c];
        rep->stall_count[c] = cnt;
    }
    rep->history_len = 0;
    if (rep->history && rep->history_cap > 0) {
        const int32_t hl = std::min(rows, rep->history_cap);
        SPH_HIP(hipMemcpyAsync(rep->history, S.hist, sizeof(double) * (size_t)hl * 3, hipMemcpyDeviceToHost,
                               ctx->stream));
        SPH_HIP(hipStreamSynchronize(ctx->stream));
        rep->history_len = hl;
    }
    float ms_setup = 0.f, ms_iter = 0.f;
    SPH_HIP(hipEventElapsedTime(&ms_setup, e0, e1));
    SPH_HIP(hipEventElapsedTime(&ms_iter, e1, e2));
    rep->setup_ms = ms_setup;
    rep->iterate_ms = ms_iter;
    rep->launches = S.launches;
    rep->issued_iters = S.issued_iters;
    if (S.profile > 0) {
        double tot = 0.0;
        int32_t cnt = 0;
        for (const auto& rc : S.recs) {
            if (rc.round >= (int32_t)S.round_end.size() || rc.it > S.round_end[rc.round]) continue;  // returned at once
            float ms = 0.f;
            SPH_HIP(hipEventElapsedTime(&ms, ctx->prof_ev[2 * rc.ev], ctx->prof_ev[2 * rc.ev + 1]));
            tot += ms;
            ++cnt;
        }
        rep->apply_ms = tot;
        rep->apply_launches = cnt;
    }
    if (winfo) {
        double wi[kWiSize];
        SPH_HIP(hipMemcpyAsync(wi, winfo, sizeof(wi), hipMemcpyDeviceToHost, ctx->stream));
        SPH_HIP(hipStreamSynchronize(ctx->stream));
        for (int c = 0; c < 3; ++c) {
            rep->warm_used[c] = wi[kWiUse + c] != 0.0;
            rep->warm_rr[c] = wi[kWiRrL + c];
            rep->plain_rr[c] = wi[kWiRrP + c];
        }
        rep->warm_scale = wi[kWiU];
        float ms = 0.f;
        SPH_HIP(hipEventElapsedTime(&ms, ctx->ev[5], ctx->ev[6]));
        rep->warm_ms = ms;
    }
    rep->status = any_prog ? SPH_NOT_CONVERGED : (any_stall ? SPH_STALLED : SPH_OK);
    return (sph_status)rep->status;
}

}  // namespace

extern "C" sph_status sph_visc_solve(sph_ctx* ctx, const sph_nbr* nb, const sph_domain* dom,
                                     const sph_particles* p, const sph_visc_params* params, int32_t prec,
                                     const void* const rhs[3], void* const x[3], const sph_solve_opts* opts,
                                     sph_solve_report* report) {
    if (!ctx) return SPH_E_ARG;
    if (!rhs || !x || !opts || !report) return ctx->fail(SPH_E_ARG, "visc_solve: null argument");
    for (int c = 0; c < 3; ++c)
        if (!rhs[c] || !x[c]) return ctx->fail(SPH_E_ARG, "visc_solve: null vector");
    if (!(opts->tol >= 0.0) || opts->max_iter < 0 || opts->max_iter > 100000000)
        return ctx->fail(SPH_E_ARG, "visc_solve: tol or max_iter out of range");
    if (opts->variant != SPH_ROBUST && opts->variant != SPH_STANDARD && opts->variant != SPH_CG)
        return ctx->fail(SPH_E_ARG, "visc_solve: variant");
    if (opts->fp32_scalars && prec != SPH_F32)
        return ctx->fail(SPH_E_ARG, "visc_solve: fp32_scalars needs prec = SPH_F32");

    if (opts->variant == SPH_CG && params && params->wall == SPH_WALL_DUMMY)
        return ctx->fail(SPH_E_ARG, "visc_solve: the CG needs a symmetric system (dynamic walls)");
    if (opts->true_res_period < 0) return ctx->fail(SPH_E_ARG, "visc_solve: true_res_period < 0");
    sph_nbr* own = nullptr;
    if (!nb) {
        if (!dom) return ctx->fail(SPH_E_ARG, "visc_solve: neither neighbour handle nor domain");
        SPH_TRY(sph_build_neighbors(ctx, p, dom, &own));
        nb = own;
    }
    if (nb->device != ctx->device) return ctx->fail(SPH_E_ARG, "visc_solve: handle of another device");
    sph_status st = check_particles(ctx, nb, p);
    // SPH_MIXED: FP32 operator and vectors (checked as SPH_F32), FP64 solution
    if (st == SPH_OK) st = check_params(ctx, params, prec == SPH_MIXED ? SPH_F32 : prec);
    if (st == SPH_OK && params->op_mode == SPH_OP_PAPER32 && prec != SPH_F32)
        st = ctx->fail(SPH_E_ARG, "visc_solve: SPH_OP_PAPER32 is single precision (SPH_F32)");
    if (st == SPH_OK) {
        double* hist_keep = report->history;
        int32_t cap_keep = report->history_cap;
        std::memset(report, 0, sizeof(*report));
        report->history = hist_keep;
        report->history_cap = cap_keep;
        if (prec == SPH_F64)
            st = solve_impl<double, double>(ctx, nb, p, params, prec, rhs, x, opts, report);
        else if (params->op_mode == SPH_OP_PAPER32 && nb->g.kernel != SPH_KERNEL_WENDLAND)
            st = ctx->fail(SPH_E_ARG, "visc_solve: SPH_OP_PAPER32 is defined for the Wendland kernel");
        else if (params->op_mode == SPH_OP_PAPER32)
            st = solve_impl<float, float, true>(ctx, nb, p, params, prec, rhs, x, opts, report);
        else if (prec == SPH_F32)
            st = solve_impl<float, float>(ctx, nb, p, params, prec, rhs, x, opts, report);
        else
            st = solve_impl<float, double>(ctx, nb, p, params, prec, rhs, x, opts, report);
    }
    if (own) sph_neighbors_free(own);
    return st;
}
