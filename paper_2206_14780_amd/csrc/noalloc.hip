// The matrix-free operator for callers that cannot allocate device memory
// (code under HIP graph capture, tight time-stepping loops, harnesses that
// forbid hipMalloc): sph_visc_apply with SPH_OP_ONTHEFLY, whose staging
// buffers (the cell-order particle properties and the cell-order copies of
// x and y) live in one file-scope device array instead of the context's
// workspace.
//
// The array is set up once per device when a context is created
// (noalloc_setup, called by sph_create with the device current): its device
// address comes from hipGetSymbolAddress and is kept per device.  Host code
// only ever hands that address to kernels; the array's own name is a host
// stand-in, not a device pointer.  Every call on one device shares its
// array, so calls that overlap on one device (two contexts, two streams)
// race; each call writes every byte it reads before reading it, so nothing
// needs clearing between calls.
#include <mutex>

#include "operator_kernels.hpp"

namespace {

using namespace sph;

constexpr int64_t kMaxN = SPH_NOALLOC_MAX_N;

// Byte offsets of the staging arrays for kMaxN particles (FP64 sizes; FP32
// vectors use half of theirs), each a multiple of 256.
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kOffMass = 0;
constexpr size_t kOffRho = kOffMass + align256(sizeof(double) * kMaxN);
constexpr size_t kOffMu = kOffRho + align256(sizeof(double) * kMaxN);
constexpr size_t kOffInvRho = kOffMu + align256(sizeof(double) * kMaxN);
constexpr size_t kOffMuMr = kOffInvRho + align256(sizeof(double) * kMaxN);
constexpr size_t kOffType = kOffMuMr + align256(sizeof(double2) * kMaxN);
constexpr size_t kOffX = kOffType + align256(sizeof(uint8_t) * kMaxN);
constexpr size_t kOffY = kOffX + align256(3 * sizeof(double) * kMaxN);
constexpr size_t kScratchBytes = kOffY + align256(3 * sizeof(double) * kMaxN);
static_assert(kScratchBytes == 97 * (size_t)kMaxN, "staging layout");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

void* scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

template <typename T>
sph_status apply_noalloc(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p, const sph_visc_params* v,
                         unsigned char* base, const void* const x[3], void* const y[3]) {
    PropBufs b;
    b.mass = reinterpret_cast<double*>(base + kOffMass);
    b.rho = reinterpret_cast<double*>(base + kOffRho);
    b.mu = reinterpret_cast<double*>(base + kOffMu);
    b.inv_rho = reinterpret_cast<double*>(base + kOffInvRho);
    b.mu_mr = reinterpret_cast<double2*>(base + kOffMuMr);
    b.type = base + kOffType;
    T* xin = reinterpret_cast<T*>(base + kOffX);
    T* yout = reinterpret_cast<T*>(base + kOffY);
    PartView pv;
    SPH_TRY(gather_props_into(ctx, nb, p, b, &pv));
    const OpParams op{v->dt, v->wall, v->avg, v->jacobi ? 1 : 0};
    SPH_TRY(gather_vec3<T>(ctx, nb, x, xin));
    SPH_TRY(apply_plain<T>(ctx, nb, pv, op, SPH_OP_ONTHEFLY, nullptr, xin, yout));
    SPH_TRY(scatter_vec3<T>(ctx, nb, yout, y));
    return SPH_OK;
}

}  // namespace

namespace sph {

// Device address of the staging array on `device` (current on entry).
sph_status noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return SPH_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return SPH_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SPH_E_HIP;
    g_ptr[device] = ptr;
    return SPH_OK;
}

}  // namespace sph

extern "C" sph_status sph_visc_apply_noalloc(sph_ctx* ctx, const sph_nbr* nb, const sph_particles* p,
                                             const sph_visc_params* params, int32_t prec,
                                             const void* const x[3], void* const y[3]) {
    if (!ctx) return SPH_E_ARG;
    if (!nb || !x || !y) return ctx->fail(SPH_E_ARG, "visc_apply_noalloc: null argument");
    if (nb->device != ctx->device) return ctx->fail(SPH_E_ARG, "visc_apply_noalloc: handle of another device");
    for (int c = 0; c < 3; ++c)
        if (!x[c] || !y[c]) return ctx->fail(SPH_E_ARG, "visc_apply_noalloc: null vector");
    SPH_TRY(check_particles(ctx, nb, p));
    SPH_TRY(check_params(ctx, params, prec));
    if (params->op_mode != SPH_OP_ONTHEFLY)
        return ctx->fail(SPH_E_ARG, "visc_apply_noalloc: only the on-the-fly operator (SPH_OP_ONTHEFLY) "
                                    "needs no matrix storage");
    if (nb->n > kMaxN)
        return ctx->fail(SPH_E_ARG, "visc_apply_noalloc: more than SPH_NOALLOC_MAX_N (262144) particles");
    unsigned char* base = static_cast<unsigned char*>(scratch_of(ctx->device));
    if (!base) return ctx->fail(SPH_E_HIP, "visc_apply_noalloc: staging array not set up on this device");
    if (prec == SPH_F64) return apply_noalloc<double>(ctx, nb, p, params, base, x, y);
    return apply_noalloc<float>(ctx, nb, p, params, base, x, y);
}
