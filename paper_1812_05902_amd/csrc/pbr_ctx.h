// Private host-side state of a context, shared by the single-image API and the batch API.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <string>
#include <vector>

#include "pbr_internal.h"

struct pbr_ctx {
    int device = 0;            // -1: host-only context (validation and derived optics, no device work)
    hipStream_t stream = nullptr;
    std::string err;
    unsigned long long *counters = nullptr;  // 4 KiB device block
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> box_ev;  // pairs around each integration launch (stats only)
    // field
    bool has_field = false;
    const float4 *cells = nullptr;
    pbr_source_sum *src_sums = nullptr;    // per-source hit sums (PBR_SOURCE_SUMS), device
    const double *mie = nullptr;            // Mie intensity table (PBR_MIE), device
    double laser[3] = {1.0, 0.0, 0.0};
    int64_t src_sums_cap = 0;
    const int64_t *src_order = nullptr;     // processing order of the sources (PBR_SOURCE_ORDER), device
    int64_t src_order_n = 0;
    unsigned *brick_gmax = nullptr;        // per-brick max |grad n| (float bits), device
    unsigned char *brick_fp64 = nullptr;   // per-brick FP64 flags, device
    pbr::FieldLayout layout{};
    int64_t n_fp64_bricks = 0;
    int nx = 0, ny = 0, nz = 0;
    double origin[3] = {0, 0, 0}, spacing[3] = {0, 0, 0};
    double K = 0.0, rho_inf = 0.0;
    // optics
    bool has_optics = false;
    bool has_chain = false;                 // a general optical chain replaces the singlet
    pbr_optical_chain chain{};
    pbr_optics optics{};
    // sensor
    bool has_sensor = false;
    pbr_sensor sensor{};
    unsigned long long *accum = nullptr;
    double accum_rays = 0.0;  // rays deposited since the last clear (overflow bound)
    // per-ray state between the trace kernels
    pbr::RayState *ray_ws = nullptr;
    int64_t ray_chunk = 0;
    // exit recording
    pbr_ray_exit *rec = nullptr;
    int64_t rec_first = 0, rec_stride = 1, rec_max = 0;
    int last_max_steps = 0;
    // identity of the scene a surrogate was trained on: unique context id, and a counter bumped
    // by every change of field, optics or sensor
    uint64_t uid = 0;
    uint64_t scene_version = 0;
    // bumped by every call that changes what a trace launch reads from the context (field, optics,
    // sensor, optical chain, exit recording): batches check it before replaying their snapshot
    uint64_t param_version = 0;
    pbr_surrogate *surr = nullptr;
};

namespace pbr {
namespace host {

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct Derived {
    double n_inf, R, t, a, clear, z_sensor, M, sigma_px;
    int rfp;
};

// Records a formatted message on the context (or the creation error when c is null).
int fail(pbr_ctx *c, int code, const char *fmt, ...);
int hip_fail(pbr_ctx *c, int e, const char *what);
// Derived optics of a context whose field, optics and sensor are set (PBR_ERR_STATE otherwise).
int derive(pbr_ctx *c, Derived *d);
// Launch parameters shared by the trace and the calibration (sources and rays left empty).
void fill_params(const pbr_ctx *ctx, const Derived &d, double ds, TraceParams *out);
// Next context id (never 0).
uint64_t next_uid();
// Normalised unpolarised Mie intensity at n_angles angles over [0, pi] (pbr_mie.cpp).
bool mie_intensity_table(std::complex<double> m, double x, int n_angles, double *out);
// Chunk hook of an attached surrogate for trace chunks of up to `chunk` rays; fails with STATE
// (message on ctx) when it no longer matches the context's scene and with WORKSPACE when its
// buffers were sized for smaller chunks.
int surrogate_hook(pbr_ctx *ctx, double ds, int64_t chunk, ChunkHook *out);
// Looks up the device address of the static ray-state array of pbr_emit_and_trace_noalloc on
// `device` (current), once per device; returns the HIP error of the lookup.
int noalloc_scratch_init(int device);
// Fingerprint of the context's stored field (device checksum of the field's words; synchronises).
int field_fingerprint(pbr_ctx *ctx, uint64_t *out);
// pbr_emit_and_trace after the null-context check.  noalloc: the ray states of the chunks go to
// static_ws (the static array of this device; null when there is none), static_chunk rays at a
// time, instead of the context's trace workspace.
int emit_and_trace_impl(pbr_ctx *ctx, const float *src_dev, int64_t n_src, int32_t rays_per_src, uint64_t seed,
                        double ds, uint32_t flags, pbr_stats *stats, bool noalloc, RayState *static_ws,
                        int64_t static_chunk);

}  // namespace host

// Counts into *bad (device) the waves that saw a non-finite density value, field_prep.hip.
int launch_check_finite(const float *rho, int64_t n, unsigned long long *bad, hipStream_t stream);
// Order-independent checksum of a device buffer's 32-bit words into *out (device), field_prep.hip.
int launch_field_checksum(const void *field, size_t bytes, unsigned long long *out, hipStream_t stream);

}  // namespace pbr
