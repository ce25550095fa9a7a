// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "sph.h"
#include "issue_plan.hpp"

namespace sph {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per block of the simple per-particle kernels
constexpr int kMaxBlock = 1024;    // largest block of the row kernels
constexpr int kMaxWaves = kMaxBlock / kWave;
constexpr int kApplyMaxBlock = 256;  // largest block of the operator kernels (register budget)
constexpr int kNumXcd = 8;         // MI355X: 8 accelerator complex dies, one L2 each
constexpr double kPi = 3.14159265358979323846;
constexpr double kGaussK = 3.0;  // radius of the truncated Gaussian kernel, in units of h

// ---------------------------------------------------------------------------
// Cell grid of a neighbour handle.  Cells are at least 2h wide on every axis,
// so all neighbours of a particle lie in the 3x3x3 block of cells around it.
// ---------------------------------------------------------------------------
struct Grid {
    int32_t nc[3];      // cells per axis
    double org[3];      // lower corner (domain lo)
    double cs[3];       // cell side
    double period[3];   // period on periodic axes, 0 elsewhere
    int32_t per[3];     // periodic flags
    double h;           // smoothing length
    double cut2;        // (support radius)^2, the neighbour predicate's bound
    double inv_h, inv_h3, inv_h5;  // 1/h, 1/h^3, 1/h^5
    int32_t kernel;     // SPH_KERNEL_WENDLAND / SPH_KERNEL_GAUSSIAN
    double gauss_norm;  // w_G of the truncated Gaussian
    double gauss_tail;  // e^{-k^2}, its value at the cut
};

// One particle's position in cell order, padded to 32 bytes so that a
// neighbour candidate costs one load.
struct alignas(32) Pos4 {
    double x, y, z, pad;
};

// Device view of a neighbour handle (cell-sorted positions).
struct NbrView {
    int64_t n;
    Grid g;
    const int32_t* cell_start;  // [ncell + 1]
    const int32_t* scell;       // cell id of each sorted particle
    const Pos4* pos;            // sorted positions
};

// Per-particle operator data in cell order.
struct PartView {
    const double* mass;
    const double* rho;
    const double* mu;
    const uint8_t* type;
    const double2* mu_mr;   // (mu, mass / rho), the neighbour data of a pair weight
    const double* inv_rho;  // 1 / rho
};

struct OpParams {
    double dt;
    int32_t wall;
    int32_t avg;
    int32_t jacobi;
    // 1: the paper's single-precision matrix (cached operator only): pair
    // weights evaluated in FP32 from cell-relative FP32 positions, FP32
    // diagonal and wall normalisation by compensated sums; the matrix keeps
    // the plain diagonal per row in place of the row sum
    int32_t f32cell = 0;
};

// Sliced ELLPACK matrix, one slice = 64 consecutive rows (one wavefront).
// Entry k of row r = s*64 + l lives at slot
//   sl_ptr[s] + (k / P) * 64 P + l P + k % P,
// with P = pack_of<T>() (4 for FP32 coefficients, 1 for FP64): each lane's P
// consecutive entries are adjacent (one vector load) and the 64 lanes' packs
// of one slot group are contiguous; slice widths are multiples of P.  Columns
// are delta coded: a row's columns ascend; the row starts at column c0[r]
// and each slot adds its 16-bit step dcol (the first entry steps by 0).  A
// step that does not fit takes an escape slot (dcol = kEscape) whose
// coefficient bits hold the whole jump and which contributes nothing.  Rows
// shorter than their slice are padded with (step 0, coef 0).  The operator is
// applied in difference form, y_r = rs_r x_r + sum_k coef[r,k] (x_col - x_r),
// with rs_r the row sum of the matrix, which the structure of A fixes exactly
// (1/A_rr for a Jacobi-scaled fluid row, 1 unscaled, 2 for a dummy-wall row
// with fluid neighbours, 1 for identity rows).  The coefficient is FP64
// evaluated and rounded once to T; FP32 keeps the remainder
// lo = coefficient - (double)coef, so coef + lo carries ~48 bits for the
// FP64-accurate residual.
constexpr uint16_t kEscape = 0xFFFF;
// Slots of a lane stored together: four FP32 coefficients make one 16-byte
// load; FP64 keeps one (four measured slower there: more registers, lower
// occupancy).
template <typename T>
constexpr int pack_of() { return sizeof(T) == 4 ? 4 : 1; }

// First slot of lane l of a slice starting at slot sl, and its k-th slot.
template <typename T>
__host__ __device__ inline int64_t lane_base(int64_t sl, int64_t lane) { return sl + lane * pack_of<T>(); }
template <typename T>
__host__ __device__ inline int64_t slot_of(int64_t lbase, int32_t k) {
    constexpr int P = pack_of<T>();
    return lbase + (int64_t)(k / P) * (64 * P) + k % P;
}

template <typename T>
struct Sell {
    int64_t nslices;
    const int64_t* sl_ptr;  // [nslices + 1]
    const T* coef;          // per slot
    const uint16_t* dcol;   // per slot: column step or kEscape
    const float* lo;        // per slot, FP32 only
    const int32_t* c0;      // per row: first column (the row itself if empty)
    const T* dg;            // row sum of the (scaled) matrix, per row
    const double* rs64;     // the same row sums in FP64
};

// ---------------------------------------------------------------------------
// Solver control block in device memory.  Fields indexed [2] are double
// buffered by iteration parity: the kernel that writes slot it&1 never reads
// it, so every block of a kernel sees the values of earlier kernels only.
// ---------------------------------------------------------------------------
enum HaltReason : int32_t { kHaltNoProg = 1, kHaltPeriodic = 2, kHaltMaxIter = 4 };

// A component that the recursive residual calls converged but the FP64 true
// residual rejects is restarted at most this many times; after that it is
// reported stalled (its precision cannot reach the tolerance).
constexpr int32_t kMaxRestarts = 3;

struct Ctl {
    // written by the p-update kernel (block 0)
    double gam[2][3];     // gamma_i = r0hat . r_{i-1}
    double alphap[2][3];  // alpha'_{i-1}
    double beta[2][3];    // beta_{i-1}
    int32_t stall0[2][3]; // textbook variant: gamma_i == 0
    int32_t nres[2][3];   // failed-check restarts so far (slot it&1 written by iteration it)
    double rr_ref[2][3];  // true r.r at the last (re)start
    double rr[3];         // r.r of the last completed iteration
    double bb[3];
    double tau2[3];
    int32_t state[3];
    int32_t iter;         // iterations started
    int32_t halt;         // nonzero: every iteration kernel returns at once
    int32_t halt_reason;
    int32_t dev_checked_iter;  // last iteration checked by the p-update kernel
    // written by the s-update kernel (block 0)
    double delta[2][3];
    double alpha[2][3];
    int32_t stallA[2][3];
    // written by the close-out kernel (block 0)
    double omega[2][3];
    int32_t stallB[2][3];
    // written by the residual-check kernels (p-update block 0 or host-issued)
    double trr[3];
    double gam_restart[3];
    double rr_restart[3];
    int32_t restart[3];
    int32_t restart_iter;
    int32_t host_checked_iter;  // last iteration checked by host-issued kernels
    int32_t n_true_checks;
    int32_t n_replaced;
    int32_t nonfinite;
};

// CtlPoll (issue_plan.hpp) mirrors a contiguous run of Ctl.
static_assert(offsetof(Ctl, halt_reason) + sizeof(int32_t) - offsetof(Ctl, rr) == sizeof(CtlPoll) &&
                  offsetof(Ctl, state) - offsetof(Ctl, rr) == offsetof(CtlPoll, state) &&
                  offsetof(Ctl, halt) - offsetof(Ctl, rr) == offsetof(CtlPoll, halt),
              "CtlPoll mirrors a contiguous run of Ctl");
constexpr size_t kHostMailBytes = 256;  // two CtlPoll slots
static_assert(2 * sizeof(CtlPoll) <= kHostMailBytes, "mailbox holds two polls");

// Constants of one solve, passed by value to the iteration kernels.
struct SolveConst {
    double tol2;
    double drop;           // restart when r_true.r_true < drop * rr_ref (0 = never)
    int32_t tr_blocks;     // blocks (partials) of the true-residual kernel
    double floor_;
    int32_t max_iter;
    int32_t variant;
    int32_t true_res_period;
    int32_t force_stall_iter;
    int32_t force_stall_comp;
    int32_t hist_cap;      // rows of the device history arrays
    int32_t fp32;          // 1: every reduced inner product and every scalar rounded to FP32
};

// Launch geometry of the row kernels.
struct Launch {
    int64_t n;
    int32_t grid_apply;    // blocks of the operator kernels
    int32_t block_apply;   // threads per operator block (multiple of 64, <= kApplyMaxBlock)
    int32_t grid_stream;   // blocks of the streaming kernels
    int32_t block_stream;  // threads per streaming block
};

Launch make_launch(int64_t n);

// ---------------------------------------------------------------------------
// Device workspace: named, monotonically growing allocations of a context.
// ---------------------------------------------------------------------------
enum Slot : int {
    kMass, kRho, kMu, kType, kMuMr, kInvRho, kCnt, kCntReal, kDiag64, kWsum, kSlSize, kSlPtr, kCoef, kDcol, kC0, kDg, kLo, kRs64,
    kVecB, kVecX, kVecR, kVecRh0, kVecP, kVecAp, kVecS, kVecAs, kVecTmp, kB64,
    kPartA1, kPartA2, kPartK3, kPartChk, kCtl, kHist, kStallHist, kScanTmp,
    kApplyIn, kApplyOut, kExportCnt, kNnzCount, kMlpPart, kMlpOut, kWarmS, kWarmO, kWarmInfo, kWarmPart,
    kWarmPart2, kWarmU, kList, kWList, kNbrCell, kNbrCount, kNbrFill, kViscU, kStepBuf, kNumSlots
};

}  // namespace sph

struct sph_ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    void* ws[sph::kNumSlots] = {};
    size_t ws_bytes[sph::kNumSlots] = {};
    void* host_mail = nullptr;   // pinned host mailbox for polling the control block
    hipEvent_t ev[7] = {};        // 0-2: solve timing, 3-4: halt polls, 5-6: learned start
    std::vector<hipEvent_t> prof_ev;  // pairs bracketing profiled launches

    sph_status fail(sph_status s, const std::string& what);
    sph_status hip_fail(hipError_t e, const char* what);
    // Ensure workspace slot `slot` holds at least `bytes`; on success *out
    // receives the device pointer.
    sph_status ensure(int slot, size_t bytes, void** out);
    template <typename P>
    sph_status ensure_t(int slot, size_t count, P** out) {
        void* v = nullptr;
        sph_status s = ensure(slot, count * sizeof(P), &v);
        *out = static_cast<P*>(v);
        return s;
    }
};

struct sph_nbr {
    int32_t device = 0;
    int64_t n = 0;
    int64_t ncell = 0;
    sph::Grid g{};
    int32_t* cell_start = nullptr;
    int32_t* scell = nullptr;
    int32_t* perm = nullptr;    // sorted -> original
    int32_t* iperm = nullptr;   // original -> sorted
    sph::Pos4* pos = nullptr;
    void* blob = nullptr;       // the one device allocation holding the arrays above
    int64_t nnz = -1;           // pair count, computed on demand

    sph::NbrView view() const {
        sph::NbrView v;
        v.n = n;
        v.g = g;
        v.cell_start = cell_start;
        v.scell = scell;
        v.pos = pos;
        return v;
    }
};

#define SPH_HIP(call)                                                  \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ctx->hip_fail(e_, #call);         \
    } while (0)

#define SPH_TRY(expr)                                                  \
    do {                                                               \
        sph_status s_ = (expr);                                        \
        if (s_ != SPH_OK) return s_;                                   \
    } while (0)

#define SPH_LAUNCHED(what)                                             \
    do {                                                               \
        hipError_t e_ = hipGetLastError();                             \
        if (e_ != hipSuccess) return ctx->hip_fail(e_, what);          \
    } while (0)

namespace sph {

// Exclusive scan of `n` values into out[0..n] (out[n] = total), on the stream.
sph_status scan_i32(sph_ctx* ctx, const int32_t* in, int32_t* out, int64_t n);
sph_status scan_i64(sph_ctx* ctx, const int64_t* in, int64_t* out, int64_t n);

// Operator pieces (operator.hip).
// Cell-order copies of the particle properties (n entries each).
struct PropBufs {
    double *mass, *rho, *mu, *inv_rho;
    uint8_t* type;
    double2* mu_mr;
};
// Gathers the properties into the context workspace, or into caller-given
// buffers (gather_props_into: allocates nothing).
sph_status gather_props(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, PartView* out);
sph_status gather_props_into(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, const PropBufs& b,
                             PartView* out);
template <typename T>
sph_status gather_vec3(sph_ctx* ctx, const sph_nbr* nb, const void* const src[3], T* dst);
// The same from caller arrays of precision S into cell-order T (S = double, T = float).
template <typename S, typename T>
sph_status gather_vec3_cvt(sph_ctx* ctx, const sph_nbr* nb, const void* const src[3], T* dst);
template <typename T>
sph_status scatter_vec3(sph_ctx* ctx, const sph_nbr* nb, const T* src, void* const dst[3]);
// Builds the cached matrix; *nnz / *slots (host, optional) receive the
// off-diagonal entry count and the stored slot count.
template <typename T>
sph_status build_sell(sph_ctx* ctx, const sph_nbr* nb, const PartView& pv, const OpParams& op,
                      Sell<T>* out, const double** diag64, int64_t* nnz = nullptr,
                      int64_t* slots = nullptr);
template <typename T>
sph_status apply_plain(sph_ctx* ctx, const sph_nbr* nb, const PartView& pv, const OpParams& op,
                       int mode, const Sell<T>* sell, const T* x, T* y);
sph_status row_diag64(sph_ctx* ctx, const sph_nbr* nb, const PartView& pv, const OpParams& op,
                      const double** diag64);

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Looks up the device address of the allocation-free entry point's staging
// array on `device` (which must be current); once per device (noalloc.hip).
sph_status noalloc_setup(int device);

}  // namespace sph

// Argument checks shared by the entry points.
sph_status check_particles(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p);
sph_status check_params(sph_ctx* ctx, const sph_visc_params* v, int32_t prec);
