// The viscous operator A(dt): particle data gathers, the cached sliced-ELL
// matrix (coefficients evaluated once per call in FP64), and the operator
// kernels used by sph_visc_apply and the solver.
#include <algorithm>
#include <cstdlib>

#include "operator_kernels.hpp"

namespace sph {

static int32_t env_int(const char* name, int32_t dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    long x = std::strtol(v, nullptr, 10);
    return x > 0 ? (int32_t)x : dflt;
}

// ---------------------------------------------------------------------------
// Gathers between the caller's order and cell order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gather_props(int64_t n, const int32_t* __restrict__ perm,
                                                         const double* __restrict__ m,
                                                         const double* __restrict__ r,
                                                         const double* __restrict__ mu,
                                                         const uint8_t* __restrict__ t,
                                                         double* __restrict__ om, double* __restrict__ orr,
                                                         double* __restrict__ omu,
                                                         uint8_t* __restrict__ ot, double2* __restrict__ omr,
                                                         double* __restrict__ oir) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t o = perm[s];
    const double ms = m[o], rs = r[o];
    om[s] = ms;
    orr[s] = rs;
    const double mus = mu[o];
    omu[s] = mus;
    ot[s] = t[o];
    omr[s] = make_double2(mus, ms / rs);
    oir[s] = 1.0 / rs;
}

template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_gather_vec3(int64_t n, const int32_t* __restrict__ perm,
                                                        const S* __restrict__ a, const S* __restrict__ b,
                                                        const S* __restrict__ c, D* __restrict__ dst) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t o = perm[s];
    V3<D> v;
    v.x = (D)a[o];
    v.y = (D)b[o];
    v.z = (D)c[o];
    st3(dst, s, v);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_vec3(int64_t n, const int32_t* __restrict__ perm,
                                                         const T* __restrict__ src, T* __restrict__ a,
                                                         T* __restrict__ b, T* __restrict__ c) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t o = perm[s];
    V3<T> v = ld3(src, s);
    a[o] = v.x;
    b[o] = v.y;
    c[o] = v.z;
}

sph_status gather_props_into(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, const PropBufs& b,
                             PartView* out) {
    const int64_t n = nb->n;
    hipLaunchKernelGGL(k_gather_props, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, ctx->stream, n,
                       nb->perm, p->mass, p->rho, p->mu, p->type, b.mass, b.rho, b.mu, b.type, b.mu_mr, b.inv_rho);
    SPH_LAUNCHED("k_gather_props");
    out->mass = b.mass;
    out->rho = b.rho;
    out->mu = b.mu;
    out->type = b.type;
    out->mu_mr = b.mu_mr;
    out->inv_rho = b.inv_rho;
    return SPH_OK;
}

sph_status gather_props(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, PartView* out) {
    const int64_t n = nb->n;
    PropBufs b;
    SPH_TRY(ctx->ensure_t(kMass, n, &b.mass));
    SPH_TRY(ctx->ensure_t(kRho, n, &b.rho));
    SPH_TRY(ctx->ensure_t(kMu, n, &b.mu));
    SPH_TRY(ctx->ensure_t(kType, n, &b.type));
    SPH_TRY(ctx->ensure_t(kMuMr, n, &b.mu_mr));
    SPH_TRY(ctx->ensure_t(kInvRho, n, &b.inv_rho));
    return gather_props_into(ctx, nb, p, b, out);
}

template <typename S, typename T>
sph_status gather_vec3_cvt(sph_ctx* ctx, const sph_nbr* nb, const void* const src[3], T* dst) {
    hipLaunchKernelGGL((k_gather_vec3<S, T>), dim3((unsigned)ceil_div(nb->n, kBlock)), dim3(kBlock), 0,
                       ctx->stream, nb->n, nb->perm, (const S*)src[0], (const S*)src[1], (const S*)src[2], dst);
    SPH_LAUNCHED("k_gather_vec3");
    return SPH_OK;
}
template sph_status gather_vec3_cvt<double, float>(sph_ctx*, const sph_nbr*, const void* const[3], float*);

template <typename T>
sph_status gather_vec3(sph_ctx* ctx, const sph_nbr* nb, const void* const src[3], T* dst) {
    hipLaunchKernelGGL((k_gather_vec3<T, T>), dim3((unsigned)ceil_div(nb->n, kBlock)), dim3(kBlock), 0, ctx->stream,
                       nb->n, nb->perm, (const T*)src[0], (const T*)src[1], (const T*)src[2], dst);
    SPH_LAUNCHED("k_gather_vec3");
    return SPH_OK;
}

template <typename T>
sph_status scatter_vec3(sph_ctx* ctx, const sph_nbr* nb, const T* src, void* const dst[3]) {
    hipLaunchKernelGGL(k_scatter_vec3<T>, dim3((unsigned)ceil_div(nb->n, kBlock)), dim3(kBlock), 0,
                       ctx->stream, nb->n, nb->perm, src, (T*)dst[0], (T*)dst[1], (T*)dst[2]);
    SPH_LAUNCHED("k_scatter_vec3");
    return SPH_OK;
}

template sph_status gather_vec3<float>(sph_ctx*, const sph_nbr*, const void* const[3], float*);
template sph_status gather_vec3<double>(sph_ctx*, const sph_nbr*, const void* const[3], double*);
template sph_status scatter_vec3<float>(sph_ctx*, const sph_nbr*, const float*, void* const[3]);
template sph_status scatter_vec3<double>(sph_ctx*, const sph_nbr*, const double*, void* const[3]);

// ---------------------------------------------------------------------------
// Delta-coded slots (see Sell): a step outside [0, kEscape) takes an escape
// slot carrying the whole jump.
// ---------------------------------------------------------------------------
__device__ inline bool needs_escape(int64_t step) { return step < 0 || step >= (int64_t)kEscape; }

// Coefficients are evaluated in FP64 and rounded once to T (FP32 also keeps
// the rounding remainder).
__device__ inline void sell_put(float* coef, uint16_t* dcol, float* lo, int64_t i, int32_t step, double c) {
    const float hi = (float)c;
    coef[i] = hi;
    lo[i] = (float)(c - (double)hi);
    dcol[i] = (uint16_t)step;
}
__device__ inline void sell_put(double* coef, uint16_t* dcol, float*, int64_t i, int32_t step, double c) {
    coef[i] = c;
    dcol[i] = (uint16_t)step;
}
__device__ inline void sell_escape(float* coef, uint16_t* dcol, float* lo, int64_t i, int32_t jump) {
    coef[i] = __int_as_float(jump);
    lo[i] = 0.f;
    dcol[i] = kEscape;
}
__device__ inline void sell_escape(double* coef, uint16_t* dcol, float*, int64_t i, int32_t jump) {
    coef[i] = __longlong_as_double((long long)jump);
    dcol[i] = kEscape;
}

// Writes one row's slots in order: put(col, c) per entry (columns as they
// come), then pad() up to the slice width.  c0 receives the first column.
template <typename T>
struct RowWriter {
    T* coef;
    uint16_t* dcol;
    float* lo;
    int64_t base;  // the lane's first slot
    int32_t j = 0;
    int32_t prev = 0;
    __device__ void put(int32_t col, double c) {
        if (j > 0) {
            const int64_t step = (int64_t)col - prev;
            if (needs_escape(step)) {
                sell_escape(coef, dcol, lo, slot_of<T>(base, j), (int32_t)step);
                ++j;
                prev = col;
            }
        } else {
            prev = col;
        }
        sell_put(coef, dcol, lo, slot_of<T>(base, j), col - prev, c);
        ++j;
        prev = col;
    }
    __device__ void pad(int32_t width) {
        for (; j < width; ++j) sell_put(coef, dcol, lo, slot_of<T>(base, j), 0, 0.0);
    }
};

// Slots of a row with c entries in column order: c plus one escape per step
// outside [0, kEscape).
struct SlotCounter {
    int32_t c = 0, slots = 0, prev = 0;
    __device__ void add(int32_t col) {
        if (c > 0 && needs_escape((int64_t)col - prev)) ++slots;
        ++c;
        ++slots;
        prev = col;
    }
};

// ---------------------------------------------------------------------------
// Matrix build, pass 1: slots and entries per row, FP64 diagonal, dummy-wall
// kernel sum.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_row_count(NbrView nv, PartView pv, OpParams op,
                                                      int32_t* __restrict__ cnt, int32_t* __restrict__ creal,
                                                      double* __restrict__ diag64,
                                                      double* __restrict__ wsum) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nv.n) return;
    const int32_t row = (int32_t)b;
    SlotCounter sc;
    double d = 1.0, sW = 0.0;
    if (pv.type[row] == SPH_FLUID) {
        double sw = 0.0;
        for_each_neighbor(nv, row, [&](int32_t a, double r2) {
            sw += pair_w(pv, nv.g, op.avg, row, a, r2);
            sc.add(a);
        });
        d = 1.0 + op.dt * sw;
    } else if (op.wall == SPH_WALL_DUMMY) {
        for_each_neighbor(nv, row, [&](int32_t a, double r2) {
            if (pv.type[a] != SPH_FLUID) return;
            sW += pair_W(nv.g, r2);
            sc.add(a);
        });
        if (!(sW > 0.0)) sc = SlotCounter{};
    }
    if (cnt) cnt[row] = sc.slots;
    if (creal) creal[row] = sc.c;
    diag64[row] = d;
    if (wsum) wsum[row] = sW;
}

// Slice size = 64 x (most slots of a row of the slice); nnz += entries.
__global__ __launch_bounds__(kBlock) void k_slice_size(int64_t n, int64_t nslices, int32_t pack,
                                                       const int32_t* __restrict__ cnt,
                                                       const int32_t* __restrict__ creal,
                                                       int64_t* __restrict__ size,
                                                       unsigned long long* __restrict__ nnz) {
    // each wave takes slices in turn, lane l reading row 64 s + l; nnz[0]:
    // nonzeros, the low 32 bits of nnz[1]: longest row (nonzeros), one
    // atomic of each kind per block
    __shared__ int64_t bt[kBlock / kWave];
    __shared__ int32_t bl[kBlock / kWave];
    const int lane = threadIdx.x % kWave;
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    int64_t tot = 0;
    int32_t longest = 0;
    for (int64_t s = (int64_t)blockIdx.x * nw + wid; s < nslices; s += (int64_t)gridDim.x * nw) {
        const int64_t r = s * kWave + lane;
        int32_t w = 0;
        if (r < n) {
            w = cnt[r];
            const int32_t c = creal[r];
            tot += c;
            longest = max(longest, c);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, kWave));
        if (lane == 0) size[s] = (int64_t)((w + pack - 1) / pack * pack) * kWave;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o, kWave);
        longest = max(longest, __shfl_xor(longest, o, kWave));
    }
    if (lane == 0) {
        bt[wid] = tot;
        bl[wid] = longest;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < nw; ++k) {
            tot += bt[k];
            longest = max(longest, bl[k]);
        }
        if (tot > 0) {
            atomicAdd(nnz, (unsigned long long)tot);
            atomicMax(reinterpret_cast<int32_t*>(nnz + 1), longest);
        }
    }
}

// Pass 2: write the slots (coefficients evaluated inside the scan).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_row_fill(NbrView nv, PartView pv, OpParams op,
                                                     const double* __restrict__ diag64,
                                                     const double* __restrict__ wsum,
                                                     const int64_t* __restrict__ sl_ptr, T* __restrict__ coef,
                                                     uint16_t* __restrict__ dcol, float* __restrict__ lo,
                                                     int32_t* __restrict__ c0, T* __restrict__ dg,
                                                     double* __restrict__ rs64, int64_t nslices) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nslices * kWave) return;
    const int64_t s = r / kWave;
    const int lane = (int)(r % kWave);
    const int32_t width = (int32_t)((sl_ptr[s + 1] - sl_ptr[s]) / kWave);
    RowWriter<T> wr{coef, dcol, lo, lane_base<T>(sl_ptr[s], lane)};
    if (r < nv.n) {
        const int32_t row = (int32_t)r;
        int32_t first = row;
        const double D = diag64[row];
        if (pv.type[row] == SPH_FLUID) {
            for_each_neighbor(nv, row, [&](int32_t a, double r2) {
                double aba = -op.dt * pair_w(pv, nv.g, op.avg, row, a, r2);
                double c = op.jacobi ? aba / D : aba;
                if (wr.j == 0) first = a;
                wr.put(a, c);
            });
            // row sum: (A 1)_r = 1 (eqs. diag, offdiag), scaled by 1/A_rr with Jacobi
            const double rs = op.jacobi ? 1.0 / D : 1.0;
            dg[row] = (T)rs;
            rs64[row] = rs;
        } else {
            const double sW = wsum[row];
            double rs = 1.0;
            if (op.wall == SPH_WALL_DUMMY && sW > 0.0) {
                for_each_neighbor(nv, row, [&](int32_t a, double r2) {
                    if (pv.type[a] != SPH_FLUID) return;
                    if (wr.j == 0) first = a;
                    wr.put(a, pair_W(nv.g, r2) / sW);
                });
                rs = 2.0;  // 1 + sum_a W_ra / sum_a W_ra (eq. implicit-system-dummy-full)
            }
            dg[row] = (T)rs;
            rs64[row] = rs;
        }
        c0[row] = first;
    }
    wr.pad(width);
}

// ---------------------------------------------------------------------------
// List-based matrix build (the default).
//
// k_row_scan: one thread per row runs the neighbour scan, counts entries and
//   slots and records the neighbour indices.  The lanes of a wave reach their
//   k-th neighbour at different points of the scan, so a direct store of each
//   index would scatter partial cache lines (several times the list size
//   written to HBM); each lane instead collects kChunk indices in LDS and
//   writes them as one 64-byte segment.  List layout, with cap entries per
//   row (cap / kChunk segments): entry k of row r sits at
//   ((r/64 * cap/kChunk + k/kChunk) * 64 + r%64) * kChunk + k%kChunk.
// k_row_fill_list: one lane per row of a slice, the lanes walking their
//   lists in step: the pair weights in list order (= scan order) give the
//   row sum and the FP64 diagonal and are kept, slot-major (entry k of the
//   64 rows of a slice written together); a second walk scales them into the
//   slots, which the lanes also write together.  A row with more than cap
//   neighbours keeps no list and is rescanned here.  cap is 96 for the
//   Wendland kernel (~80 neighbours) and 288 for the truncated Gaussian
//   (~250), unless the lists of a large system would not fit their budget
//   (then 96, and its rows are all rescanned).
// Same pairs, summation order and coefficients as the scan-order build.
// ---------------------------------------------------------------------------
constexpr int kChunk = 16;                    // indices per segment
constexpr int kListCap = 96;                  // listed neighbours per row, Wendland kernel
constexpr int kListCapGauss = 288;            // the same, truncated Gaussian
constexpr size_t kListBudget = size_t(24) << 30;  // bytes of lists and weights at most
constexpr int kBufStride = kChunk + 1;        // LDS words per lane (odd: no bank conflicts)
constexpr int kFillGroup = 8;                 // list entries whose gathers are issued together
static_assert(kListCap % kChunk == 0 && kListCapGauss % kChunk == 0, "whole segments");

__device__ inline int64_t list_base(int64_t r, int32_t cap) {
    return ((r / kWave) * (cap / kChunk) * kWave + (r % kWave)) * kChunk;
}
__device__ inline int64_t list_off(int32_t k) {
    return (int64_t)(k / kChunk) * (kWave * kChunk) + (k % kChunk);
}

// Row kinds: fluid rows take every neighbour, dummy-wall rows their fluid
// neighbours, other wall rows none (identity rows).
enum { kRowNone = 0, kRowFluid = 1, kRowDummy = 2 };
__device__ inline int row_kind(const PartView& pv, const OpParams& op, int32_t row) {
    if (pv.type[row] == SPH_FLUID) return kRowFluid;
    return op.wall == SPH_WALL_DUMMY ? kRowDummy : kRowNone;
}

__global__ __launch_bounds__(kBlock) void k_row_scan(NbrView nv, PartView pv, OpParams op,
                                                     int32_t* __restrict__ cnt, int32_t* __restrict__ creal,
                                                     int32_t* __restrict__ list, int32_t cap) {
    __shared__ int32_t buf[kBlock * kBufStride];
    const int64_t b = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (b >= nv.n) return;  // (each lane uses only its own LDS words)
    const int32_t row = (int32_t)b;
    int32_t* my = buf + threadIdx.x * kBufStride;
    int32_t* out = list + list_base(b, cap);
    const auto flush = [&](int32_t q) {
        int4* dst = reinterpret_cast<int4*>(out + (int64_t)q * (kWave * kChunk));
#pragma unroll
        for (int i = 0; i < kChunk / 4; ++i)
            dst[i] = make_int4(my[4 * i], my[4 * i + 1], my[4 * i + 2], my[4 * i + 3]);
    };
    SlotCounter sc;
    const auto push = [&](int32_t a) {
        const int32_t e = sc.c % kChunk;
        my[e] = a;
        if (e == kChunk - 1 && sc.c < cap) flush(sc.c / kChunk);
        sc.add(a);
    };
    const int kind = row_kind(pv, op, row);
    if (kind == kRowFluid) {
        for_each_neighbor(nv, row, [&](int32_t a, double) { push(a); });
    } else if (kind == kRowDummy) {
        for_each_neighbor(nv, row, [&](int32_t a, double) {
            if (pv.type[a] == SPH_FLUID) push(a);
        });
    }
    if (sc.c <= cap && sc.c % kChunk) flush(sc.c / kChunk);
    cnt[row] = sc.slots;
    creal[row] = sc.c;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_row_fill_list(NbrView nv, PartView pv, OpParams op, int64_t nslices,
                                                          const int32_t* __restrict__ creal,
                                                          const int32_t* __restrict__ list,
                                                          double* __restrict__ wlist,
                                                          const int64_t* __restrict__ sl_ptr, T* __restrict__ coef,
                                                          uint16_t* __restrict__ dcol, float* __restrict__ lo,
                                                          int32_t* __restrict__ c0, T* __restrict__ dg,
                                                          double* __restrict__ rs64, double* __restrict__ diag64,
                                                          int32_t cap) {
    const int64_t r = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (r >= nslices * kWave) return;
    const Grid& g = nv.g;
    const int64_t s = r / kWave;
    const bool valid = r < nv.n;
    const int32_t row = valid ? (int32_t)r : 0;
    const int kind = valid ? row_kind(pv, op, row) : kRowNone;
    int32_t c = kind != kRowNone ? creal[row] : 0;
    const bool listed = c <= cap;
    const int32_t* lst = list + list_base(r, cap);
    double* wl = wlist + (r / kWave) * ((int64_t)cap * kWave) + r % kWave;  // entry k at wl[k * kWave]
    const Pos4 pb = nv.pos[row];
    const double mu_b = pv.mu[row], ir_b = pv.inv_rho[row];
    const bool f32 = op.f32cell != 0;
    const auto weight = [&](int32_t a, double r2) {
        if (kind != kRowFluid) return pair_W(g, r2);
        const double2 ma = pv.mu_mr[a];
        return pair_w_v(g, op.avg, ma.x, ma.y, mu_b, ir_b, r2);
    };
    // the paper's single precision: FP32 weight from cell-relative positions
    const int32_t cb = nv.scell[row];
    const float mub32 = (float)mu_b, rhob32 = (float)pv.rho[row];
    const auto weight32 = [&](int32_t a) -> double {
        const float r2 = dist2_f32(g, pb, cb, nv.pos[a], nv.scell[a]);
        if (kind != kRowFluid) return (double)wendland_W_f32(g, r2);
        return (double)pair_w_f32(g, op.avg, (float)pv.mu[a], (float)pv.mass[a], (float)pv.rho[a], mub32, rhob32,
                                  r2);
    };
    const auto scan = [&](auto&& f) {  // unlisted rows: the scan again
        for_each_neighbor(nv, row, [&](int32_t a, double r2) {
            if (kind == kRowDummy && pv.type[a] != SPH_FLUID) return;
            f(a, r2);
        });
    };
    double sum = 0.0;
    float sum32 = 0.f, cmp32 = 0.f;  // compensated FP32 sum (f32)
    const auto add = [&](double w) {
        if (f32) kahan_add(sum32, cmp32, (float)w);
        else sum += w;
    };
    if (listed && !f32) {
        // groups of kFillGroup entries: indices, then positions and
        // neighbour data loaded together, then the weights in list order
        for (int32_t k0 = 0; k0 < c; k0 += kFillGroup) {
            int32_t a[kFillGroup];
#pragma unroll
            for (int u = 0; u < kFillGroup; ++u) a[u] = k0 + u < c ? lst[list_off(k0 + u)] : row;
            Pos4 pa[kFillGroup];
            double2 ma[kFillGroup];
#pragma unroll
            for (int u = 0; u < kFillGroup; ++u) pa[u] = nv.pos[a[u]];
            if (kind == kRowFluid) {
#pragma unroll
                for (int u = 0; u < kFillGroup; ++u) ma[u] = pv.mu_mr[a[u]];
            }
#pragma unroll
            for (int u = 0; u < kFillGroup; ++u) {
                if (k0 + u >= c) break;
                // r^2 exactly as the scan computes it
                const double dx = disp(pb.x, pa[u].x, g.period[0]);
                const double dy = disp(pb.y, pa[u].y, g.period[1]);
                const double dz = disp(pb.z, pa[u].z, g.period[2]);
                const double r2 = (dx * dx + dy * dy) + dz * dz;
                const double w = kind != kRowFluid ? pair_W(g, r2)
                                                   : pair_w_v(g, op.avg, ma[u].x, ma[u].y, mu_b, ir_b, r2);
                wl[(k0 + u) * kWave] = w;
                add(w);
            }
        }
    } else if (listed) {
        for (int32_t k = 0; k < c; ++k) {
            const int32_t a = lst[list_off(k)];
            const double w = weight32(a);
            wl[k * kWave] = w;
            add(w);
        }
    } else {
        scan([&](int32_t a, double r2) { add(f32 ? weight32(a) : weight(a, r2)); });
    }
    if (f32) sum = (double)sum32;
    const float D32 = kind == kRowFluid ? 1.0f + (float)op.dt * sum32 : 1.0f;
    const double D = f32 ? (double)D32 : (kind == kRowFluid ? 1.0 + op.dt * sum : 1.0);
    if (kind == kRowDummy && !(sum > 0.0)) c = 0;  // identity row
    const auto coefficient = [&](double w) {
        if (f32) {
            if (kind == kRowFluid) {
                const float aba = -((float)op.dt * (float)w);
                return (double)(op.jacobi ? aba / D32 : aba);
            }
            return (double)((float)w / sum32);
        }
        if (kind == kRowFluid) {
            const double aba = -op.dt * w;
            return op.jacobi ? aba / D : aba;
        }
        return w / sum;
    };
    const int32_t width = (int32_t)((sl_ptr[s + 1] - sl_ptr[s]) / kWave);
    RowWriter<T> wr{coef, dcol, lo, lane_base<T>(sl_ptr[s], r % kWave)};
    int32_t first = row;
    double csum = 0.0;  // f32: FP64 sum of the stored coefficients
    if (listed) {
        for (int32_t k = 0; k < c; ++k) {
            const int32_t a = lst[list_off(k)];
            if (k == 0) first = a;
            const double cv = coefficient(wl[k * kWave]);
            csum += cv;
            wr.put(a, cv);
        }
    } else if (c > 0) {
        scan([&](int32_t a, double r2) {
            if (wr.j == 0) first = a;
            const double cv = coefficient(f32 ? weight32(a) : weight(a, r2));
            csum += cv;
            wr.put(a, cv);
        });
    }
    wr.pad(width);
    if (valid) {
        c0[row] = first;
        if (f32) {
            // the plain diagonal A_rr (1 when scaled, on identity and on
            // dummy rows); the FP64 row sum of the stored FP32 matrix for
            // the difference form of the true residual
            const double dd = kind == kRowFluid && !op.jacobi ? D : 1.0;
            dg[row] = (T)dd;
            rs64[row] = dd + csum;
        } else {
            // row sums: 1/A_rr (Jacobi) or 1 on fluid rows (eqs. diag, offdiag),
            // 2 on dummy rows with fluid neighbours (eq. implicit-system-dummy-full),
            // 1 on identity rows
            const double rs = kind == kRowFluid ? (op.jacobi ? 1.0 / D : 1.0) : (c > 0 ? 2.0 : 1.0);
            dg[row] = (T)rs;
            rs64[row] = rs;
        }
        diag64[row] = D;
    }
}

sph_status row_diag64(sph_ctx* ctx, const sph_nbr* nb, const PartView& pv, const OpParams& op,
                      const double** diag64) {
    double* d = nullptr;
    SPH_TRY(ctx->ensure_t(kDiag64, nb->n, &d));
    hipLaunchKernelGGL(k_row_count, dim3((unsigned)ceil_div(nb->n, kBlock)), dim3(kBlock), 0, ctx->stream,
                       nb->view(), pv, op, (int32_t*)nullptr, (int32_t*)nullptr, d, (double*)nullptr);
    SPH_LAUNCHED("k_row_count");
    *diag64 = d;
    return SPH_OK;
}

template <typename T>
sph_status build_sell(sph_ctx* ctx, const sph_nbr* nb, const PartView& pv, const OpParams& op, Sell<T>* out,
                      const double** diag64, int64_t* nnz_out, int64_t* slots_out) {
    const int64_t n = nb->n;
    const int64_t nslices = ceil_div(n, kWave);
    // Test hook: the environment variable SPH_BUILD_LEGACY=1 selects the
    // build that evaluates the coefficients inside the neighbour scan, the
    // reference the list-based build is tested against bit for bit.
    if (op.f32cell && nb->g.kernel != SPH_KERNEL_WENDLAND)
        return ctx->fail(SPH_E_ARG, "SPH_OP_PAPER32 is defined for the Wendland kernel");
    const bool legacy = env_int("SPH_BUILD_LEGACY", 0) > 0 && !op.f32cell;
    // list entries per row: room for every neighbour of the kernel's support
    // (int32 index + FP64 weight each) while that fits the budget
    const int32_t cap = nb->g.kernel == SPH_KERNEL_GAUSSIAN &&
                                (size_t)nslices * kWave * kListCapGauss * 12 <= kListBudget
                            ? kListCapGauss
                            : kListCap;
    int32_t *cnt = nullptr, *creal = nullptr, *list = nullptr;
    double *d = nullptr, *ws = nullptr, *wlist = nullptr;
    int64_t *size = nullptr, *ptr = nullptr;
    SPH_TRY(ctx->ensure_t(kCnt, n, &cnt));
    SPH_TRY(ctx->ensure_t(kCntReal, n, &creal));
    SPH_TRY(ctx->ensure_t(kDiag64, n, &d));
    SPH_TRY(ctx->ensure_t(kSlSize, nslices, &size));
    SPH_TRY(ctx->ensure_t(kSlPtr, nslices + 1, &ptr));
    unsigned long long* nnz_dev = nullptr;  // [0] nonzeros, [1] longest row
    SPH_TRY(ctx->ensure_t(kNnzCount, 2, &nnz_dev));
    SPH_HIP(hipMemsetAsync(nnz_dev, 0, 2 * sizeof(unsigned long long), ctx->stream));
    // row kernels: whole XCD rounds of blocks (xcd_block needs a multiple of 8)
    const dim3 rows_grid((unsigned)(ceil_div(ceil_div(n, kBlock), kNumXcd) * kNumXcd));
    const dim3 slice_grid((unsigned)(ceil_div(ceil_div(nslices * kWave, kBlock), kNumXcd) * kNumXcd));
    if (legacy) {
        SPH_TRY(ctx->ensure_t(kWsum, n, &ws));
        hipLaunchKernelGGL(k_row_count, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, ctx->stream,
                           nb->view(), pv, op, cnt, creal, d, ws);
    } else {
        SPH_TRY(ctx->ensure_t(kList, (size_t)nslices * cap * kWave, &list));
        SPH_TRY(ctx->ensure_t(kWList, (size_t)nslices * cap * kWave, &wlist));
        hipLaunchKernelGGL(k_row_scan, rows_grid, dim3(kBlock), 0, ctx->stream, nb->view(), pv, op, cnt, creal,
                           list, cap);
    }
    hipLaunchKernelGGL(k_slice_size, dim3((unsigned)std::min<int64_t>(ceil_div(nslices * kWave, kBlock), 1024)),
                       dim3(kBlock), 0, ctx->stream,
                       n, nslices, (int32_t)pack_of<T>(), cnt, creal, size, nnz_dev);
    SPH_LAUNCHED("k_row_count/k_slice_size");
    SPH_TRY(scan_i64(ctx, size, ptr, nslices));
    int64_t nnzp = 0;
    unsigned long long hcnt[2] = {0, 0};
    SPH_HIP(hipMemcpyAsync(&nnzp, ptr + nslices, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    SPH_HIP(hipMemcpyAsync(hcnt, nnz_dev, sizeof(hcnt), hipMemcpyDeviceToHost, ctx->stream));
    SPH_HIP(hipStreamSynchronize(ctx->stream));
    if (nnz_out) *nnz_out = (int64_t)hcnt[0];
    if (slots_out) *slots_out = nnzp;
    T* coef = nullptr;
    uint16_t* dcol = nullptr;
    float* lo = nullptr;
    int32_t* c0 = nullptr;
    T* dg = nullptr;
    const size_t ns = (size_t)(nnzp > 0 ? nnzp : 1);
    SPH_TRY(ctx->ensure_t(kCoef, ns, &coef));
    SPH_TRY(ctx->ensure_t(kDcol, ns, &dcol));
    if constexpr (sizeof(T) == 4) SPH_TRY(ctx->ensure_t(kLo, ns, &lo));
    SPH_TRY(ctx->ensure_t(kC0, n, &c0));
    double* rs64 = nullptr;
    SPH_TRY(ctx->ensure_t(kDg, n, &dg));
    SPH_TRY(ctx->ensure_t(kRs64, n, &rs64));
    if (!legacy) {
        // Occupancy limit: the launch reserves LDS it does not use, so that
        // only two blocks share a CU.  The neighbour gathers of the rows in
        // flight on an XCD then fit its L2 (with eight blocks per CU they
        // did not): 8.1 -> 5.8 ms at 4.49M particles.
        constexpr size_t kFillLdsReserve = 60 * 1024;
        hipLaunchKernelGGL(k_row_fill_list<T>, slice_grid, dim3(kBlock), kFillLdsReserve, ctx->stream, nb->view(), pv, op,
                           nslices, creal, list, wlist, ptr, coef, dcol, lo, c0, dg, rs64, d, cap);
        SPH_LAUNCHED("k_row_fill_list");
    } else {
        hipLaunchKernelGGL(k_row_fill<T>, dim3((unsigned)ceil_div(nslices * kWave, kBlock)), dim3(kBlock), 0,
                           ctx->stream, nb->view(), pv, op, d, ws, ptr, coef, dcol, lo, c0, dg, rs64, nslices);
        SPH_LAUNCHED("k_row_fill");
    }
    out->nslices = nslices;
    out->sl_ptr = ptr;
    out->coef = coef;
    out->dcol = dcol;
    out->lo = lo;
    out->c0 = c0;
    out->dg = dg;
    out->rs64 = rs64;
    if (diag64) *diag64 = d;
    return SPH_OK;
}

template sph_status build_sell<float>(sph_ctx*, const sph_nbr*, const PartView&, const OpParams&, Sell<float>*,
                                      const double**, int64_t*, int64_t*);
template sph_status build_sell<double>(sph_ctx*, const sph_nbr*, const PartView&, const OpParams&,
                                       Sell<double>*, const double**, int64_t*, int64_t*);


// Launch geometry of the row kernels.
Launch make_launch(int64_t n) {
    Launch L;
    L.n = n;
    const int64_t nslices = ceil_div(n, kWave);
    const int32_t ba = kApplyMaxBlock;
    const int64_t wpb = ba / kWave;
    // one 64-row slice per wave: the launch's tail is then one slice long
    // (measured fastest for whole iterations on the 1.16M and 4.49M tanks);
    // the grid is rounded up to a multiple of the XCD count, so that no block
    // gets more slices than it has waves
    int64_t ga = ceil_div(nslices, wpb);
    if (ga >= 64) ga = ceil_div(ga, kNumXcd) * kNumXcd;
    L.grid_apply = (int32_t)std::max<int64_t>(ga, 1);
    L.block_apply = ba;
    // streaming kernels: every block re-reduces the previous kernel's
    // partials, so each thread should stream at least 8 rows of the (at most
    // 256-block) grid: the largest power-of-two block up to 1024 that keeps
    // that (512 at N = 1.16M, 1024 from N = 2.1M; measured 28.8 against
    // 29.3 ms per step on the 1.16M tank, no change at 4.7M)
    int32_t bs_def = 1024;
    while (bs_def > kWave && (int64_t)bs_def * 256 * 8 > n) bs_def /= 2;
    const int32_t bs = bs_def;
    int64_t gs = std::min<int64_t>(ceil_div(n, (int64_t)bs * 4), 256);
    if (gs >= 64) gs = gs / kNumXcd * kNumXcd;
    L.grid_stream = (int32_t)std::max<int64_t>(gs, 1);
    L.block_stream = bs;
    return L;
}

template <typename T>
sph_status apply_plain(sph_ctx* ctx, const sph_nbr* nb, const PartView& pv, const OpParams& op, int mode,
                       const Sell<T>* sell, const T* x, T* y) {
    const Launch L = make_launch(nb->n);
    if (mode == SPH_OP_PAPER32) {
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((k_apply_sell<T, kDotNone, T, true>), dim3(L.grid_apply), dim3(L.block_apply), 0,
                               ctx->stream, (const int32_t*)nullptr, nb->n, *sell, x, y, (const T*)nullptr,
                               (const double*)nullptr, (double*)nullptr);
        else
            return ctx->fail(SPH_E_ARG, "apply: SPH_OP_PAPER32 is single precision");
    } else if (mode == SPH_OP_CACHED) {
        hipLaunchKernelGGL((k_apply_sell<T, kDotNone>), dim3(L.grid_apply), dim3(L.block_apply), 0, ctx->stream,
                           (const int32_t*)nullptr, nb->n, *sell, x, y, (const T*)nullptr, (const double*)nullptr,
                           (double*)nullptr);
    } else {
        hipLaunchKernelGGL((k_apply_otf<T, kDotNone>), dim3(L.grid_apply), dim3(L.block_apply), 0, ctx->stream,
                           (const int32_t*)nullptr, nb->view(), pv, op, x, y, (const T*)nullptr,
                           (const double*)nullptr, (double*)nullptr);
    }
    SPH_LAUNCHED("apply");
    return SPH_OK;
}

template sph_status apply_plain<float>(sph_ctx*, const sph_nbr*, const PartView&, const OpParams&, int,
                                       const Sell<float>*, const float*, float*);
template sph_status apply_plain<double>(sph_ctx*, const sph_nbr*, const PartView&, const OpParams&, int,
                                        const Sell<double>*, const double*, double*);

}  // namespace sph

using namespace sph;

sph_status check_particles(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p) {
    if (!p) return ctx->fail(SPH_E_ARG, "null particles");
    if (p->n != nb->n) return ctx->fail(SPH_E_ARG, "particle count differs from the neighbour handle");
    if (!p->mass || !p->rho || !p->mu || !p->type) return ctx->fail(SPH_E_ARG, "null particle array");
    return SPH_OK;
}

sph_status check_params(sph_ctx* ctx, const sph_visc_params* v, int32_t prec) {
    if (!v) return ctx->fail(SPH_E_ARG, "null params");
    if (!(v->dt >= 0.0) || !std::isfinite(v->dt)) return ctx->fail(SPH_E_ARG, "params: dt must be finite and >= 0");
    if (v->wall != SPH_WALL_DYNAMIC && v->wall != SPH_WALL_DUMMY) return ctx->fail(SPH_E_ARG, "params: wall");
    if (v->avg != SPH_AVG_ARITH && v->avg != SPH_AVG_HARMONIC) return ctx->fail(SPH_E_ARG, "params: avg");
    if (v->op_mode != SPH_OP_CACHED && v->op_mode != SPH_OP_ONTHEFLY && v->op_mode != SPH_OP_PAPER32)
        return ctx->fail(SPH_E_ARG, "params: op_mode");
    if (prec != SPH_F32 && prec != SPH_F64) return ctx->fail(SPH_E_ARG, "prec");
    if (v->op_mode == SPH_OP_PAPER32 && prec != SPH_F32)
        return ctx->fail(SPH_E_ARG, "params: SPH_OP_PAPER32 is single precision (SPH_F32)");
    return SPH_OK;
}

template <typename T>
static sph_status apply_entry(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p,
                              const sph_visc_params* v, const void* const x[3], void* const y[3]) {
    PartView pv;
    SPH_TRY(gather_props(ctx, nb, p, &pv));
    OpParams op{v->dt, v->wall, v->avg, v->jacobi ? 1 : 0};
    T *xin = nullptr, *yout = nullptr;
    SPH_TRY(ctx->ensure_t(kApplyIn, (size_t)nb->n * 3, &xin));
    SPH_TRY(ctx->ensure_t(kApplyOut, (size_t)nb->n * 3, &yout));
    SPH_TRY(gather_vec3<T>(ctx, nb, x, xin));
    Sell<T> sell{};
    if (v->op_mode == SPH_OP_PAPER32) op.f32cell = 1;
    if (v->op_mode != SPH_OP_ONTHEFLY) SPH_TRY(build_sell<T>(ctx, nb, pv, op, &sell, nullptr));
    SPH_TRY(apply_plain<T>(ctx, nb, pv, op, v->op_mode, &sell, xin, yout));
    SPH_TRY(scatter_vec3<T>(ctx, nb, yout, y));
    return SPH_OK;
}

extern "C" sph_status sph_visc_apply(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p,
                                     const sph_visc_params* params, int32_t prec, const void* const x[3],
                                     void* const y[3]) {
    if (!ctx) return SPH_E_ARG;
    if (!nb || !x || !y) return ctx->fail(SPH_E_ARG, "visc_apply: null argument");
    if (nb->device != ctx->device) return ctx->fail(SPH_E_ARG, "visc_apply: handle of another device");
    for (int c = 0; c < 3; ++c)
        if (!x[c] || !y[c]) return ctx->fail(SPH_E_ARG, "visc_apply: null vector");
    SPH_TRY(check_particles(ctx, nb, p));
    SPH_TRY(check_params(ctx, params, prec));
    if (prec == SPH_F64) return apply_entry<double>(ctx, nb, p, params, x, y);
    return apply_entry<float>(ctx, nb, p, params, x, y);
}
