// Context management, workspace, status strings.
#include <cstdio>

#include "sph_internal.hpp"

sph_status sph_ctx::fail(sph_status s, const std::string& what) {
    err = what;
    return s;
}

sph_status sph_ctx::hip_fail(hipError_t e, const char* what) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
    err = buf;
    return e == hipErrorOutOfMemory ? SPH_E_OOM : SPH_E_HIP;
}

sph_status sph_ctx::ensure(int slot, size_t bytes, void** out) {
    if (bytes == 0) bytes = 1;
    if (ws_bytes[slot] < bytes) {
        if (ws[slot]) {
            // the buffer may still be read by queued work
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(ws[slot]);
            ws[slot] = nullptr;
            ws_bytes[slot] = 0;
        }
        size_t grow = bytes + bytes / 8;
        hipError_t e = hipMalloc(&ws[slot], grow);
        if (e != hipSuccess) {
            ws[slot] = nullptr;
            return hip_fail(e, "hipMalloc (workspace)");
        }
        ws_bytes[slot] = grow;
    }
    *out = ws[slot];
    return SPH_OK;
}

extern "C" sph_status sph_create(sph_ctx** out, int32_t device, void* hip_stream) {
    if (!out) return SPH_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SPH_E_HIP;
    if (device < 0 || device >= ndev) return SPH_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return SPH_E_HIP;
    if (sph::noalloc_setup(device) != SPH_OK) return SPH_E_HIP;
    sph_ctx* ctx = new sph_ctx();
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    if (hipHostMalloc(&ctx->host_mail, sph::kHostMailBytes, hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return SPH_E_OOM;
    }
    for (auto& e : ctx->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            sph_destroy(ctx);
            return SPH_E_HIP;
        }
    }
    *out = ctx;
    return SPH_OK;
}

extern "C" sph_status sph_destroy(sph_ctx* ctx) {
    if (!ctx) return SPH_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < sph::kNumSlots; ++i)
        if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->prof_ev) (void)hipEventDestroy(e);
    if (ctx->host_mail) (void)hipHostFree(ctx->host_mail);
    delete ctx;
    return SPH_OK;
}

extern "C" sph_status sph_set_stream(sph_ctx* ctx, void* hip_stream) {
    if (!ctx) return SPH_E_ARG;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return SPH_OK;
}

extern "C" const char* sph_last_error(const sph_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" const char* sph_status_str(sph_status s) {
    switch (s) {
        case SPH_OK: return "ok";
        case SPH_STALLED: return "stalled";
        case SPH_NOT_CONVERGED: return "not converged";
        case SPH_E_ARG: return "invalid argument";
        case SPH_E_OOM: return "out of device memory";
        case SPH_E_HIP: return "HIP runtime error";
        case SPH_E_OVERFLOW: return "output capacity too small";
        case SPH_E_NONFINITE: return "non-finite input";
    }
    return "unknown status";
}
