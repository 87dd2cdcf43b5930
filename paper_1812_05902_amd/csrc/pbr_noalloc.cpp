// pbr_emit_and_trace_noalloc: the trace of pbr_emit_and_trace with the per-ray state of each
// chunk held in a static device array instead of the context's trace workspace, so that the call
// allocates no device memory (for callers under stream capture or in loops that must not allocate).
//
// The array lives in this file's device code object: every GPU the library runs on holds its own
// copy (PBR_NOALLOC_MAX_CHUNK rays x 64 B) until the process ends.  Host code never passes the
// array's name to a kernel: its device address is looked up once per device with
// hipGetSymbolAddress (at pbr_create, with that device current) and only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pbr_ctx.h"

namespace {

constexpr int kMaxDevices = 64;

// Ray states of one trace chunk; only ever reached through the per-device address below.
__device__ __align__(256) pbr::RayState scratch[PBR_NOALLOC_MAX_CHUNK];

std::mutex g_mu;
pbr::RayState *g_ptr[kMaxDevices] = {};
int g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

namespace pbr {
namespace host {

int noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_done[device]) return g_err[device];
    void *p = nullptr;
    const int e = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e) (void)hipGetLastError();
    g_done[device] = true;
    g_err[device] = e;
    g_ptr[device] = e ? nullptr : (pbr::RayState *)p;
    return e;
}

}  // namespace host
}  // namespace pbr

extern "C" int pbr_emit_and_trace_noalloc(pbr_ctx *ctx, const float *src_dev, int64_t n_src, int32_t rays_per_src,
                                          uint64_t seed, double ds, uint32_t flags, int64_t rays_per_chunk,
                                          pbr_stats *stats)
{
    using namespace pbr::host;
    if (!ctx) return PBR_ERR_ARG;
    try {
        if (rays_per_chunk == 0) rays_per_chunk = PBR_NOALLOC_MAX_CHUNK;
        if (rays_per_chunk < 256 || rays_per_chunk > PBR_NOALLOC_MAX_CHUNK)
            return fail(ctx, PBR_ERR_ARG,
                        "rays_per_chunk %lld outside [256, %d] (the static ray-state array holds %d rays; 0 takes all)",
                        (long long)rays_per_chunk, PBR_NOALLOC_MAX_CHUNK, PBR_NOALLOC_MAX_CHUNK);
        pbr::RayState *ws = nullptr;
        if (ctx->device >= 0 && ctx->device < kMaxDevices) {
            std::lock_guard<std::mutex> lk(g_mu);
            if (g_done[ctx->device] && g_err[ctx->device])
                return fail(ctx, PBR_ERR_HIP, "static ray-state array of device %d: %s", ctx->device,
                            hipGetErrorString((hipError_t)g_err[ctx->device]));
            ws = g_ptr[ctx->device];
        }
        return emit_and_trace_impl(ctx, src_dev, n_src, rays_per_src, seed, ds, flags, stats, true, ws,
                                   rays_per_chunk);
    } catch (...) {
        return fail(ctx, PBR_ERR_HIP, "internal error (exception)");
    }
}
