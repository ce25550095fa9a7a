// Cell-linked neighbour structure by counting sort, device prefix sums, and
// the canonical neighbour-list export.
#include <cmath>

#include "sph_device.hpp"

namespace sph {

// ---------------------------------------------------------------------------
// Exclusive prefix sum: out[i] = sum_{j<i} in[j], out[n] = total.
// Three passes: per-block scan of 1024 values, scan of the block totals by a
// single block, add-back.
// ---------------------------------------------------------------------------
constexpr int kScanPer = 4;
constexpr int kScanTile = kBlock * kScanPer;

template <typename I>
__device__ inline I block_exclusive_scan(I v, I* lds, I* total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    I inc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        I t = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += t;
    }
    if (lane == kWave - 1) lds[wid] = inc;
    __syncthreads();
    I wave_off = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
        if (w < wid) wave_off += lds[w];
        tot += lds[w];
    }
    __syncthreads();
    *total = tot;
    return wave_off + inc - v;
}

template <typename I>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const I* __restrict__ in, I* __restrict__ out,
                                                       I* __restrict__ tile_sum, int64_t n) {
    __shared__ I lds[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    I v[kScanPer];
    I s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = (base + k < n) ? in[base + k] : I(0);
        s += v[k];
    }
    I total;
    I off = block_exclusive_scan<I>(s, lds, &total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = off;
        off += v[k];
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

template <typename I>
__global__ __launch_bounds__(1024) void k_scan_sums(I* __restrict__ tile_sum, int64_t ntiles,
                                                    I* __restrict__ out_total) {
    __shared__ I lds[1024 / kWave];
    I carry = 0;
    for (int64_t b0 = 0; b0 < ntiles; b0 += blockDim.x) {
        int64_t i = b0 + threadIdx.x;
        I v = i < ntiles ? tile_sum[i] : I(0);
        I total;
        I ex = block_exclusive_scan<I>(v, lds, &total);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *out_total = carry;
}

template <typename I>
__global__ __launch_bounds__(kBlock) void k_scan_add(I* __restrict__ out, const I* __restrict__ tile_sum,
                                                     int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    const I add = tile_sum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) out[base + k] += add;
}

template <typename I>
static sph_status scan_impl(sph_ctx* ctx, const I* in, I* out, int64_t n) {
    if (n <= 0) {
        SPH_HIP(hipMemsetAsync(out, 0, sizeof(I), ctx->stream));
        return SPH_OK;
    }
    const int64_t ntiles = ceil_div(n, kScanTile);
    I* tiles = nullptr;
    SPH_TRY(ctx->ensure_t(kScanTmp, (size_t)ntiles, &tiles));
    hipLaunchKernelGGL(k_scan_tiles<I>, dim3((unsigned)ntiles), dim3(kBlock), 0, ctx->stream, in, out,
                       tiles, n);
    hipLaunchKernelGGL(k_scan_sums<I>, dim3(1), dim3(1024), 0, ctx->stream, tiles, ntiles, out + n);
    hipLaunchKernelGGL(k_scan_add<I>, dim3((unsigned)ntiles), dim3(kBlock), 0, ctx->stream, out, tiles,
                       n);
    SPH_LAUNCHED("scan");
    return SPH_OK;
}

sph_status scan_i32(sph_ctx* ctx, const int32_t* in, int32_t* out, int64_t n) {
    return scan_impl<int32_t>(ctx, in, out, n);
}
sph_status scan_i64(sph_ctx* ctx, const int64_t* in, int64_t* out, int64_t n) {
    return scan_impl<int64_t>(ctx, in, out, n);
}

// ---------------------------------------------------------------------------
// Counting sort of particles into cells.
// ---------------------------------------------------------------------------
__device__ inline int32_t cell_axis(double v, double org, double cs, int32_t nc, int32_t per) {
    double u = floor((v - org) / cs);
    int64_t c;
    if (!(u == u)) c = 0;  // NaN position: first cell (the predicate rejects it anyway)
    else if (u < -1e15) c = -1000000000LL;
    else if (u > 1e15) c = 1000000000LL;
    else c = (int64_t)u;
    if (per) {
        c %= nc;
        if (c < 0) c += nc;
    } else {
        if (c < 0) c = 0;
        if (c >= nc) c = nc - 1;
    }
    return (int32_t)c;
}

__global__ __launch_bounds__(kBlock) void k_cell_of(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ z, Grid g,
                                                    int32_t* __restrict__ cell,
                                                    int32_t* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t cx = cell_axis(x[i], g.org[0], g.cs[0], g.nc[0], g.per[0]);
    const int32_t cy = cell_axis(y[i], g.org[1], g.cs[1], g.nc[1], g.per[1]);
    const int32_t cz = cell_axis(z[i], g.org[2], g.cs[2], g.nc[2], g.per[2]);
    const int32_t c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
    cell[i] = c;
    atomicAdd(&count[c], 1);
}

__global__ __launch_bounds__(kBlock) void k_scatter(int64_t n, const int32_t* __restrict__ cell,
                                                    const int32_t* __restrict__ cell_start,
                                                    int32_t* __restrict__ fill,
                                                    int32_t* __restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = cell[i];
    const int32_t slot = cell_start[c] + atomicAdd(&fill[c], 1);
    perm[slot] = (int32_t)i;
}

// The scatter above leaves each cell in arrival order; sort every cell by
// original index so the layout is deterministic.
__global__ __launch_bounds__(kBlock) void k_sort_cells(int64_t ncell,
                                                       const int32_t* __restrict__ cell_start,
                                                       int32_t* __restrict__ perm) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int32_t b = cell_start[c], e = cell_start[c + 1];
    for (int32_t i = b + 1; i < e; ++i) {
        int32_t v = perm[i];
        int32_t j = i - 1;
        while (j >= b && perm[j] > v) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_gather_pos(int64_t n, const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ cell,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ z,
                                                       Pos4* __restrict__ pos,
                                                       int32_t* __restrict__ scell,
                                                       int32_t* __restrict__ iperm) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t o = perm[s];
    pos[s] = Pos4{x[o], y[o], z[o], 0.0};
    scell[s] = cell[o];
    iperm[o] = (int32_t)s;
}

// ---------------------------------------------------------------------------
// Canonical export: CSR over original indices, columns ascending.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_count_orig(NbrView nv, const int32_t* __restrict__ iperm,
                                                       int64_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv.n) return;
    int64_t c = 0;
    for_each_neighbor(nv, iperm[i], [&](int32_t, double) { ++c; });
    cnt[i] = c;
}

__global__ __launch_bounds__(kBlock) void k_fill_orig(NbrView nv, const int32_t* __restrict__ iperm,
                                                      const int32_t* __restrict__ perm,
                                                      const int64_t* __restrict__ row_ptr,
                                                      int32_t* __restrict__ cols) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv.n) return;
    const int64_t b = row_ptr[i];
    int64_t k = b;
    for_each_neighbor(nv, iperm[i], [&](int32_t a, double) { cols[k++] = perm[a]; });
    for (int64_t u = b + 1; u < k; ++u) {
        int32_t v = cols[u];
        int64_t j = u - 1;
        while (j >= b && cols[j] > v) {
            cols[j + 1] = cols[j];
            --j;
        }
        cols[j + 1] = v;
    }
}

}  // namespace sph

using namespace sph;

static sph_status make_grid(sph_ctx* ctx, const sph_domain* dom, Grid* g, int64_t* ncell) {
    if (!(dom->h > 0.0) || !std::isfinite(dom->h)) return ctx->fail(SPH_E_ARG, "domain: h must be > 0");
    if (dom->kernel != SPH_KERNEL_WENDLAND && dom->kernel != SPH_KERNEL_GAUSSIAN)
        return ctx->fail(SPH_E_ARG, "domain: kernel");
    g->kernel = dom->kernel;
    // support radius: 2h (Wendland) or k h with k = 3 (truncated Gaussian)
    const double s = (dom->kernel == SPH_KERNEL_GAUSSIAN ? kGaussK : 2.0) * dom->h;
    g->gauss_tail = std::exp(-kGaussK * kGaussK);
    g->gauss_norm = std::pow(kPi, 1.5) * std::erf(kGaussK) -
                    2.0 * kPi / 3.0 * std::exp(-kGaussK * kGaussK) * kGaussK * (3.0 + 2.0 * kGaussK * kGaussK);
    g->h = dom->h;
    g->cut2 = s * s;
    g->inv_h = 1.0 / dom->h;
    g->inv_h3 = g->inv_h * g->inv_h * g->inv_h;
    g->inv_h5 = g->inv_h3 * g->inv_h * g->inv_h;
    int64_t total = 1;
    for (int a = 0; a < 3; ++a) {
        double L = dom->hi[a] - dom->lo[a];
        if (!std::isfinite(L) || !(L >= 0.0)) return ctx->fail(SPH_E_ARG, "domain: hi < lo");
        g->per[a] = dom->periodic[a] ? 1 : 0;
        g->org[a] = dom->lo[a];
        // cells a hair wider than the support, so that rounding in the binning can never
        // separate two neighbours by more than one cell
        double target = s * (1.0 + 1e-9);
        int64_t nc = (int64_t)std::floor(L / target);
        if (g->per[a]) {
            if (!(L > 0.0)) return ctx->fail(SPH_E_ARG, "domain: periodic axis of zero length");
            if (nc < 1) nc = 1;
            g->period[a] = L;
        } else {
            if (nc < 1) nc = 1;
            g->period[a] = 0.0;
        }
        if (nc > (1 << 20)) return ctx->fail(SPH_E_ARG, "domain: too many cells on one axis");
        g->nc[a] = (int32_t)nc;
        g->cs[a] = L > 0.0 ? L / (double)nc : 1.0;
        if (!g->per[a] && nc == 1) g->cs[a] = L > 0.0 ? 2.0 * L : 1.0;
        total *= nc;
    }
    if (total > (int64_t)INT32_MAX / 2) return ctx->fail(SPH_E_ARG, "domain: too many cells");
    *ncell = total;
    return SPH_OK;
}

extern "C" sph_status sph_build_neighbors(sph_ctx* ctx, const sph_particles* p, const sph_domain* dom,
                                          sph_nbr** out) {
    if (!ctx) return SPH_E_ARG;
    if (!p || !dom || !out) return ctx->fail(SPH_E_ARG, "build_neighbors: null argument");
    if (p->n < 1 || p->n >= INT32_MAX) return ctx->fail(SPH_E_ARG, "build_neighbors: n out of range");
    if (!p->x || !p->y || !p->z) return ctx->fail(SPH_E_ARG, "build_neighbors: null position array");
    *out = nullptr;
    Grid g{};
    int64_t ncell = 0;
    SPH_TRY(make_grid(ctx, dom, &g, &ncell));
    const int64_t n = p->n;

    sph_nbr* nb = new sph_nbr();
    nb->device = ctx->device;
    nb->n = n;
    nb->ncell = ncell;
    nb->g = g;
    // temporaries from the context's workspace; the handle's arrays in one
    // allocation (device allocations and frees cost tens of microseconds each)
    int32_t *cell = nullptr, *count = nullptr, *fill = nullptr;
    auto fail_oom = [&]() {
        sph_neighbors_free(nb);
        return ctx->fail(SPH_E_OOM, "build_neighbors: device allocation failed");
    };
    {
        const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t b_cs = up(sizeof(int32_t) * (size_t)(ncell + 1)), b_i = up(sizeof(int32_t) * (size_t)n);
        const size_t b_pos = up(sizeof(Pos4) * (size_t)n);
        char* base = nullptr;
        if (hipMalloc(&base, b_cs + 3 * b_i + b_pos) != hipSuccess) return fail_oom();
        nb->blob = base;
        nb->cell_start = reinterpret_cast<int32_t*>(base);
        nb->scell = reinterpret_cast<int32_t*>(base + b_cs);
        nb->perm = reinterpret_cast<int32_t*>(base + b_cs + b_i);
        nb->iperm = reinterpret_cast<int32_t*>(base + b_cs + 2 * b_i);
        nb->pos = reinterpret_cast<Pos4*>(base + b_cs + 3 * b_i);
    }
    {
        sph_status st = ctx->ensure_t(kNbrCell, (size_t)n, &cell);
        if (st == SPH_OK) st = ctx->ensure_t(kNbrCount, (size_t)ncell, &count);
        if (st == SPH_OK) st = ctx->ensure_t(kNbrFill, (size_t)ncell, &fill);
        if (st != SPH_OK) {
            sph_neighbors_free(nb);
            return st;
        }
    }

    hipError_t e = hipSuccess;
    auto hip_err = [&](const char* what) {
        sph_neighbors_free(nb);
        return ctx->hip_fail(e, what);
    };
    if ((e = hipMemsetAsync(count, 0, sizeof(int32_t) * ncell, ctx->stream)) != hipSuccess) return hip_err("memset");
    if ((e = hipMemsetAsync(fill, 0, sizeof(int32_t) * ncell, ctx->stream)) != hipSuccess) return hip_err("memset");
    const unsigned gp = (unsigned)ceil_div(n, kBlock);
    const unsigned gc = (unsigned)ceil_div(ncell, kBlock);
    hipLaunchKernelGGL(k_cell_of, dim3(gp), dim3(kBlock), 0, ctx->stream, n, p->x, p->y, p->z, g, cell, count);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err("k_cell_of");
    sph_status st = scan_i32(ctx, count, nb->cell_start, ncell);
    if (st != SPH_OK) {
        sph_neighbors_free(nb);
        return st;
    }
    hipLaunchKernelGGL(k_scatter, dim3(gp), dim3(kBlock), 0, ctx->stream, n, cell, nb->cell_start, fill, nb->perm);
    hipLaunchKernelGGL(k_sort_cells, dim3(gc), dim3(kBlock), 0, ctx->stream, ncell, nb->cell_start, nb->perm);
    hipLaunchKernelGGL(k_gather_pos, dim3(gp), dim3(kBlock), 0, ctx->stream, n, nb->perm, cell, p->x, p->y,
                       p->z, nb->pos, nb->scell, nb->iperm);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err("neighbour build kernels");
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_err("hipStreamSynchronize");
    *out = nb;
    return SPH_OK;
}

static sph_status count_pairs(sph_ctx* ctx, const sph_nbr* nb, int64_t** cnt_out) {
    int64_t* cnt = nullptr;
    SPH_TRY(ctx->ensure_t(kExportCnt, (size_t)(nb->n + 1), &cnt));
    hipLaunchKernelGGL(k_count_orig, dim3((unsigned)ceil_div(nb->n, kBlock)), dim3(kBlock), 0, ctx->stream,
                       nb->view(), nb->iperm, cnt);
    SPH_LAUNCHED("k_count_orig");
    *cnt_out = cnt;
    return SPH_OK;
}

extern "C" sph_status sph_neighbors_info(sph_ctx* ctx, const sph_nbr* nb, int64_t* n, int64_t* nnz) {
    if (!ctx) return SPH_E_ARG;
    if (!nb || !n || !nnz) return ctx->fail(SPH_E_ARG, "neighbors_info: null argument");
    if (nb->device != ctx->device) return ctx->fail(SPH_E_ARG, "neighbors_info: handle of another device");
    *n = nb->n;
    if (nb->nnz < 0) {
        int64_t* cnt = nullptr;
        SPH_TRY(count_pairs(ctx, nb, &cnt));
        int64_t* rp = nullptr;
        SPH_TRY(ctx->ensure_t(kApplyOut, (size_t)(nb->n + 1), &rp));
        SPH_TRY(scan_i64(ctx, cnt, rp, nb->n));
        int64_t total = 0;
        SPH_HIP(hipMemcpyAsync(&total, rp + nb->n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
        SPH_HIP(hipStreamSynchronize(ctx->stream));
        const_cast<sph_nbr*>(nb)->nnz = total;
    }
    *nnz = nb->nnz;
    return SPH_OK;
}

extern "C" sph_status sph_neighbors_export(sph_ctx* ctx, const sph_nbr* nb, int64_t* row_ptr, int32_t* cols,
                                           int64_t cap, int64_t* nnz) {
    if (!ctx) return SPH_E_ARG;
    if (!nb || !row_ptr || !nnz) return ctx->fail(SPH_E_ARG, "neighbors_export: null argument");
    if (nb->device != ctx->device) return ctx->fail(SPH_E_ARG, "neighbors_export: handle of another device");
    int64_t* cnt = nullptr;
    SPH_TRY(count_pairs(ctx, nb, &cnt));
    SPH_TRY(scan_i64(ctx, cnt, row_ptr, nb->n));
    int64_t total = 0;
    SPH_HIP(hipMemcpyAsync(&total, row_ptr + nb->n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    SPH_HIP(hipStreamSynchronize(ctx->stream));
    const_cast<sph_nbr*>(nb)->nnz = total;
    *nnz = total;
    if (total > cap || (!cols && total > 0)) return ctx->fail(SPH_E_OVERFLOW, "neighbors_export: cols too small");
    hipLaunchKernelGGL(k_fill_orig, dim3((unsigned)ceil_div(nb->n, kBlock)), dim3(kBlock), 0, ctx->stream,
                       nb->view(), nb->iperm, nb->perm, row_ptr, cols);
    SPH_LAUNCHED("k_fill_orig");
    SPH_HIP(hipStreamSynchronize(ctx->stream));
    return SPH_OK;
}

extern "C" sph_status sph_neighbors_free(sph_nbr* nb) {
    if (!nb) return SPH_OK;
    (void)hipFree(nb->blob);
    delete nb;
    return SPH_OK;
}
