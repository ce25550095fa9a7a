// Device-side building blocks: kernel function, neighbour traversal, pair
// coefficients, vector access and wavefront/block reductions.
#pragma once

#include "sph_internal.hpp"

namespace sph {

// Wendland psi_{3,1} kernel of radius 2 (Section "Smoothing kernel choice"):
// W(r,h) = w(r/h)/h^3 with w(q) = 21/(16 pi) (1 - q/2)^4 (2q + 1), and
// F(r,h) = (1/r) dW/dr = f(r/h)/h^5 with f(q) = 105/(128 pi) (q - 2)^3, both
// zero for q >= 2.
__device__ inline double wendland_w(double q) {
    if (!(q < 2.0)) return 0.0;
    double a = 1.0 - 0.5 * q;
    return 21.0 / (16.0 * kPi) * (a * a * a * a) * (2.0 * q + 1.0);
}

__device__ inline double wendland_f(double q) {
    if (!(q < 2.0)) return 0.0;
    double a = q - 2.0;
    return 105.0 / (128.0 * kPi) * (a * a * a);
}

// Normalised truncated Gaussian of radius k = 3 (Section "Smoothing kernel
// choice"): w(q) = (e^{-q^2} - e^{-k^2}) / w_G and f(q) = w'(q)/q =
// -2 e^{-q^2} / w_G for q < k (the derivative's sign, as for the Wendland f).
__device__ inline double gauss_w(const Grid& g, double q) {
    if (!(q < kGaussK)) return 0.0;
    return (exp(-q * q) - g.gauss_tail) / g.gauss_norm;
}

__device__ inline double gauss_f(const Grid& g, double q) {
    if (!(q < kGaussK)) return 0.0;
    return -2.0 * exp(-q * q) / g.gauss_norm;
}

// The handle's kernel: w(q) and f(q) (W = w/h^3, F = f/h^5).
__device__ inline double kernel_w(const Grid& g, double q) {
    return g.kernel == SPH_KERNEL_GAUSSIAN ? gauss_w(g, q) : wendland_w(q);
}
__device__ inline double kernel_f(const Grid& g, double q) {
    return g.kernel == SPH_KERNEL_GAUSSIAN ? gauss_f(g, q) : wendland_f(q);
}

// Displacement on one axis, minimum image on periodic axes:
// d - period * rint(d / period) with d = xb - xa, the same everywhere in the
// library (contraction off), so that every path agrees on which pairs are
// neighbours.  The quotient needs no division below one period: rounding is
// monotonic, so |d| <= period/2 (exact in binary) gives |fl(d/period)| <= 1/2
// and rint 0 (ties to even); period/2 < |d| < period gives a quotient above
// 1/2 + 2^-54 (the next double above period/2 is at least that far), which
// rounds above 1/2 and to at most 1, so rint gives sign(d) and the product
// is exactly +-period.  Only |d| >= period takes the division.
__device__ inline double disp(double xb, double xa, double period) {
    double d = xb - xa;
    if (period > 0.0) {
        const double a = fabs(d);
        if (a > 0.5 * period) d = a < period ? d - copysign(period, d) : d - period * rint(d / period);
    }
    return d;
}

// 2 * mean viscosity: arithmetic (mu_a + mu_b), harmonic 4 mu_a mu_b/(mu_a + mu_b)
// (Section "Discretized equations").
__device__ inline double two_mubar(double ma, double mb, int avg) {
    if (avg == SPH_AVG_HARMONIC) {
        double s = ma + mb;
        return s > 0.0 ? 4.0 * (ma * mb) / s : 0.0;
    }
    return ma + mb;
}

// Distinct cells of the {c-1, c, c+1} block along one axis, ascending
// (periodic axes with fewer than three cells visit each of their cells once).
__device__ inline int axis_cells(int32_t c, int32_t n, int32_t per, int32_t (&out)[3]) {
    if (per) {
        if (n >= 3) {
            if (c == 0) {
                out[0] = 0; out[1] = 1; out[2] = n - 1;
            } else if (c == n - 1) {
                out[0] = 0; out[1] = n - 2; out[2] = n - 1;
            } else {
                out[0] = c - 1; out[1] = c; out[2] = c + 1;
            }
            return 3;
        }
        for (int i = 0; i < n; ++i) out[i] = i;
        return n;
    }
    int m = 0;
    for (int d = -1; d <= 1; ++d)
        if (c + d >= 0 && c + d < n) out[m++] = c + d;
    return m;
}

// Calls f(a, r2) for every neighbour a of sorted particle `row` (a != row,
// r2 = |r_row - r_a|^2 < (2h)^2), visiting the 3x3x3 cell block around the
// particle's cell as at most 9 runs of consecutive cells along x (a wrapped
// periodic x adds a second run), in ascending cell order, so that neighbours
// come in ascending index order.
template <class F>
__device__ inline void for_each_neighbor(const NbrView& nv, int32_t row, F&& f) {
    const Grid& g = nv.g;
    const Pos4 pb = nv.pos[row];
    const double xb = pb.x, yb = pb.y, zb = pb.z;
    const int32_t c = nv.scell[row];
    const int32_t nx = g.nc[0], ny = g.nc[1];
    const int32_t cx = c % nx;
    const int32_t cy = (c / nx) % ny;
    const int32_t cz = c / (nx * ny);
    int32_t zs[3], ys[3];
    const int nzs = axis_cells(cz, g.nc[2], g.per[2], zs);
    const int nys = axis_cells(cy, ny, g.per[1], ys);
    // x runs [a0, b0] and [a1, b1] (second run empty unless x wraps)
    int32_t a0, b0, a1 = 1, b1 = 0;
    if (g.per[0] && nx >= 3) {
        if (cx == 0) { a0 = 0; b0 = 1; a1 = nx - 1; b1 = nx - 1; }
        else if (cx == nx - 1) { a0 = 0; b0 = 0; a1 = nx - 2; b1 = nx - 1; }
        else { a0 = cx - 1; b0 = cx + 1; }
    } else if (g.per[0]) {
        a0 = 0; b0 = nx - 1;
    } else {
        a0 = cx > 0 ? cx - 1 : 0;
        b0 = cx < nx - 1 ? cx + 1 : nx - 1;
    }
    for (int iz = 0; iz < nzs; ++iz) {
        for (int iy = 0; iy < nys; ++iy) {
            const int32_t base = (zs[iz] * ny + ys[iy]) * nx;
            for (int run = 0; run < 2; ++run) {
                const int32_t xa = run == 0 ? a0 : a1;
                const int32_t xe = run == 0 ? b0 : b1;
                if (xa > xe) continue;
                const int32_t beg = nv.cell_start[base + xa];
                const int32_t end = nv.cell_start[base + xe + 1];
                for (int32_t a = beg; a < end; ++a) {
                    if (a == row) continue;
                    const Pos4 pa = nv.pos[a];
                    double dx = disp(xb, pa.x, g.period[0]);
                    double dy = disp(yb, pa.y, g.period[1]);
                    double dz = disp(zb, pa.z, g.period[2]);
                    double r2 = (dx * dx + dy * dy) + dz * dz;
                    if (r2 < g.cut2) f(a, r2);
                }
            }
        }
    }
}

// Pair weight w_ba = -2 mubar m_a F(r)/(rho_a rho_b) >= 0 of row b and
// neighbour a (eq. kab, diffusive sign), from the precomputed m_a/rho_a,
// 1/rho_b and powers of 1/h (one division left: the harmonic mean).
__device__ inline double pair_w_v(const Grid& g, int avg, double mu_a, double mr_a, double mu_b, double ir_b,
                                  double r2) {
    const double q = sqrt(r2) * g.inv_h;
    const double F = kernel_f(g, q) * g.inv_h5;
    const double tm = two_mubar(mu_a, mu_b, avg);
    return -(tm * mr_a * F) * ir_b;
}
__device__ inline double pair_w(const PartView& pv, const Grid& g, int avg, int32_t b,
                                int32_t a, double r2) {
    const double2 ma = pv.mu_mr[a];
    return pair_w_v(g, avg, ma.x, ma.y, pv.mu[b], pv.inv_rho[b], r2);
}

// Kernel value W_ba of the dummy-wall rows (eq. dummyvel).
__device__ inline double pair_W(const Grid& g, double r2) {
    const double q = sqrt(r2) * g.inv_h;
    return kernel_w(g, q) * g.inv_h3;
}

// ---------------------------------------------------------------------------
// Single-precision pair data from cell-relative positions (appendix on
// relative positions): each particle's position is held as its FP32 offset
// r' from the centre of its cell, and the displacement of a pair is
// o' + (r'_b - r'_a) with o' = l (c_b - c_a) the FP32 offset of the two cell
// centres (the grouping that rounds the same way for (b, a) and (a, b), so
// the matrix stays numerically symmetric where it should).  The cell offset
// is the minimum image: on periodic axes the integer cell difference takes
// the period multiple that the FP64 displacement of the neighbour search
// takes.
// ---------------------------------------------------------------------------
__device__ inline int32_t cell_coord(const Grid& g, int32_t c, int axis) {
    if (axis == 0) return c % g.nc[0];
    if (axis == 1) return (c / g.nc[0]) % g.nc[1];
    return c / (g.nc[0] * g.nc[1]);
}
// FP32 offset of coordinate x from the centre of cell index ci on an axis.
__device__ inline float rel_pos(const Grid& g, int axis, double x, int32_t ci) {
    const double centre = g.org[axis] + ((double)ci + 0.5) * g.cs[axis];
    return (float)disp(x, centre, g.period[axis]);
}
// FP32 squared distance of sorted particles b and a from cell-relative data.
__device__ inline float dist2_f32(const Grid& g, const Pos4& pb, int32_t cb, const Pos4& pa, int32_t ca) {
    const double xb[3] = {pb.x, pb.y, pb.z}, xa[3] = {pa.x, pa.y, pa.z};
    float d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t ib = cell_coord(g, cb, k), ia = cell_coord(g, ca, k);
        const float rb = rel_pos(g, k, xb[k], ib), ra = rel_pos(g, k, xa[k], ia);
        int64_t dc = (int64_t)ib - ia;
        if (g.period[k] > 0.0) {
            const double d64 = disp(xb[k], xa[k], g.period[k]);
            const double rest = d64 - (double)dc * g.cs[k] - ((double)rb - (double)ra);
            dc += (int64_t)rint(rest / g.period[k]) * g.nc[k];
        }
        const float o = (float)g.cs[k] * (float)dc;
        d[k] = o + (rb - ra);
    }
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}
// Wendland F(r) = f(r/h)/h^5 and W(r) = w(r/h)/h^3 in FP32.
__device__ inline float wendland_F_f32(const Grid& g, float r2) {
    const float q = sqrtf(r2) / (float)g.h;
    if (!(q < 2.0f)) return 0.0f;
    const float a = q - 2.0f;
    return ((float)(105.0 / (128.0 * kPi)) * ((a * a) * a)) * (float)g.inv_h5;
}
__device__ inline float wendland_W_f32(const Grid& g, float r2) {
    const float q = sqrtf(r2) / (float)g.h;
    if (!(q < 2.0f)) return 0.0f;
    const float a = 1.0f - 0.5f * q;
    return (((float)(21.0 / (16.0 * kPi)) * (((a * a) * a) * a)) * (2.0f * q + 1.0f)) * (float)g.inv_h3;
}
// Pair weight of eq. kab in FP32: -(2 mubar m_a / rho_a) F / rho_b.
__device__ inline float pair_w_f32(const Grid& g, int avg, float mu_a, float m_a, float rho_a, float mu_b,
                                   float rho_b, float r2) {
    float tm;
    if (avg == SPH_AVG_HARMONIC) {
        const float s = mu_a + mu_b;
        tm = s > 0.0f ? (4.0f * (mu_a * mu_b)) / s : 0.0f;
    } else {
        tm = mu_a + mu_b;
    }
    const float F = wendland_F_f32(g, r2);
    return -((tm * (m_a / rho_a)) * F) / rho_b;
}

// ---------------------------------------------------------------------------
// Interleaved 3-vectors (x, y, z of one particle adjacent in memory).
// ---------------------------------------------------------------------------
template <typename T>
struct V3 {
    T x, y, z;
};

template <typename T>
__device__ inline V3<T> ld3(const T* __restrict__ v, int64_t i) {
    V3<T> r;
    r.x = v[3 * i + 0];
    r.y = v[3 * i + 1];
    r.z = v[3 * i + 2];
    return r;
}

template <typename T>
__device__ inline void st3(T* __restrict__ v, int64_t i, V3<T> a) {
    v[3 * i + 0] = a.x;
    v[3 * i + 1] = a.y;
    v[3 * i + 2] = a.z;
}

__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// Reductions.  Every sum is taken in a fixed order that depends only on the
// launch geometry, so repeated runs give bitwise identical scalars.
// ---------------------------------------------------------------------------
// A double moved across lanes by DPP (CTRL: a GFX9 DPP control word), both
// halves; every source lane lies in the same row of 16, so none is masked.
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline double read_lane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// Sum over the 64 lanes of a wavefront with DPP lane moves (no LDS
// traffic): a butterfly inside each row of 16 lanes (swap neighbours, swap
// pairs, mirror the half rows, mirror the row), after which every lane of a
// row holds the same row sum (each addition sees the same two operands in
// both lanes), then the four row sums read from lanes 15, 31, 47 and 63 and
// added as (R0 + R1) + (R2 + R3).  The result is the same in every lane.
__device__ inline double wave_sum(double v) {
    v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    return (read_lane(v, 15) + read_lane(v, 31)) + (read_lane(v, 47) + read_lane(v, 63));
}

// Block-wide sum of K values per thread; result valid in every thread.
// `lds` must hold K * kMaxWaves doubles.
template <int K>
__device__ inline void block_sum(double (&v)[K], double* lds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[k * kMaxWaves + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[k * kMaxWaves + w];
        v[k] = s;
    }
    __syncthreads();
}

// Sums K partials per block written by a previous kernel:
// part[blk * K + k], blk < nblk.  Every block computes the same result.
template <int K>
__device__ inline void reduce_partials(const double* __restrict__ part, int nblk, double (&out)[K],
                                       double* lds) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] += part[(int64_t)b * K + k];
    }
    block_sum<K>(out, lds);
}

// Writes the block's K sums as its partials (thread 0).
template <int K>
__device__ inline void write_partials(double (&v)[K], double* lds, double* __restrict__ part) {
    block_sum<K>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) part[(int64_t)blockIdx.x * K + k] = v[k];
    }
}

__device__ inline bool finite_d(double v) { return __builtin_isfinite(v); }

// ---------------------------------------------------------------------------
// Compensated single-precision sums: the paper's arithmetic for every
// multi-term sum in single precision (Kahan's summation; appendix
// "Implementation notes").  A running sum is the pair (s, c): s the FP32
// sum, c Kahan's compensation (the rounding error of the last addition,
// subtracted from the next term).  Each lane sums its own terms in order;
// lanes, waves and blocks are merged by adding the other sum's s and then
// its -c the same way, in a fixed order.  Every block's merged sum s is its
// partial; the next kernel's blocks sum the partials again with Kahan's
// compensation, thread by thread in block order, then merge.
// ---------------------------------------------------------------------------
__device__ inline void kahan_add(float& s, float& c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}
__device__ inline void kahan_merge(float& s, float& c, float s2, float c2) {
    kahan_add(s, c, s2);
    kahan_add(s, c, -c2);
}

// One term of an inner product: acc += a b in FP64 (KH false) or the FP32
// product of a and b added with compensation (KH true: acc holds the FP32
// sum exactly, comp its compensation).
template <bool KH>
__device__ inline void dot_add(double& acc, float& comp, double a, double b) {
    if constexpr (!KH) {
        acc += a * b;
    } else {
        float s = (float)acc;
        kahan_add(s, comp, (float)a * (float)b);
        acc = (double)s;
    }
}
// (w a) b with each product rounded to FP32 under KH.
template <bool KH>
__device__ inline void dot_add_w(double& acc, float& comp, double w, double a, double b) {
    if constexpr (!KH) {
        acc += w * a * b;
    } else {
        float s = (float)acc;
        kahan_add(s, comp, ((float)w * (float)a) * (float)b);
        acc = (double)s;
    }
}

// Block-wide compensated merge of K per-thread sums; result (FP32 values)
// valid in every thread.  `lds` must hold 2 K kMaxWaves doubles.
template <int K>
__device__ inline void block_sum_kahan(double (&v)[K], float (&cmp)[K], double* lds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    float s[K], c[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        s[k] = (float)v[k];
        c[k] = cmp[k];
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float s2 = __shfl_xor(s[k], off, kWave);
            const float c2 = __shfl_xor(c[k], off, kWave);
            // the lower lane of each pair keeps its own sum first, so both
            // lanes form the same merged value
            if (lane & off) {
                float a = s2, b = c2;
                kahan_merge(a, b, s[k], c[k]);
                s[k] = a;
                c[k] = b;
            } else {
                kahan_merge(s[k], c[k], s2, c2);
            }
        }
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            lds[(2 * k) * kMaxWaves + wid] = (double)s[k];
            lds[(2 * k + 1) * kMaxWaves + wid] = (double)c[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float a = 0.f, b = 0.f;
        for (int w = 0; w < nw; ++w)
            kahan_merge(a, b, (float)lds[(2 * k) * kMaxWaves + w], (float)lds[(2 * k + 1) * kMaxWaves + w]);
        v[k] = (double)a;
        cmp[k] = b;
    }
    __syncthreads();
}

// Partials of the block: FP64 sums (KH false) or merged Kahan sums.
template <int K, bool KH>
__device__ inline void write_partials_kh(double (&v)[K], float (&cmp)[K], double* lds,
                                         double* __restrict__ part) {
    if constexpr (!KH) {
        write_partials<K>(v, lds, part);
    } else {
        block_sum_kahan<K>(v, cmp, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) part[(int64_t)blockIdx.x * K + k] = v[k];
        }
    }
}

// reduce_partials, or (KH) the compensated FP32 sum of the partials.
template <int K, bool KH>
__device__ inline void reduce_partials_kh(const double* __restrict__ part, int nblk, double (&out)[K],
                                          double* lds) {
    if constexpr (!KH) {
        reduce_partials<K>(part, nblk, out, lds);
    } else {
        float cmp[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            float s = 0.f, c = 0.f;
            for (int b = threadIdx.x; b < nblk; b += blockDim.x) kahan_add(s, c, (float)part[(int64_t)b * K + k]);
            out[k] = (double)s;
            cmp[k] = c;
        }
        block_sum_kahan<K>(out, cmp, lds);
    }
}

// XCD-aware block order: the hardware hands consecutive block ids to the 8
// XCDs in turn; remap so that each XCD works on one contiguous share of the
// rows and its L2 keeps the neighbour data of that share.
__device__ inline int32_t xcd_block(int32_t b, int32_t nblk) {
    const int32_t per = nblk / kNumXcd;
    if (per == 0 || nblk % kNumXcd) return b;
    return (b % kNumXcd) * per + b / kNumXcd;
}

}  // namespace sph
