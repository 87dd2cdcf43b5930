// C ABI of the library (include/pbr.h): argument validation, host-side optics set-up and the
// launches on the context's stream.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pbr_ctx.h"
#include "piv_internal.h"

namespace pbr {
namespace host {

thread_local std::string g_create_err;

int fail(pbr_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_err = buf;
    return code;
}

int hip_fail(pbr_ctx *c, int e, const char *what)
{
    return fail(c, PBR_ERR_HIP, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Host-side optics: lens radii from the thick-lens lensmaker equation (R1 = -R2 = R, glass index
// relative to vacuum), the paraxial system matrix of the lens in the ambient medium, the image
// plane of z_focus and the lateral magnification, and the spot sigma from eq. 8.
int derive(pbr_ctx *c, Derived *d)
{
    if (!c->has_field || !(c->has_optics || c->has_chain) || !c->has_sensor)
        return fail(c, PBR_ERR_STATE, "field, optics and sensor must be set first");
    const pbr_optics &o = c->optics;
    const pbr_sensor &s = c->sensor;
    d->n_inf = 1.0 + c->K * c->rho_inf;
    if (c->has_chain) {
        // a general chain has no singlet: explicit sensor plane and spot
        if (!std::isfinite(s.z_sensor) || !(s.sigma_px > 0.0))
            return fail(c, PBR_ERR_STATE, "an optical chain needs an explicit sensor plane and sigma_px > 0");
        d->R = d->t = d->clear = d->M = std::nan("");
        d->a = c->chain.aim_radius;
        d->z_sensor = s.z_sensor;
        d->sigma_px = s.sigma_px;
        d->rfp = std::max(1, (int)std::ceil(3.0 * d->sigma_px));
        if (d->rfp > pbr::kMaxFootprint)
            return fail(c, PBR_ERR_ARG, "spot sigma %.3g px needs a window wider than %d px", d->sigma_px,
                        2 * pbr::kMaxFootprint + 1);
        return PBR_OK;
    }
    const double f = o.focal_length, ng = o.n_glass;
    d->t = o.thickness > 0.0 ? o.thickness : 0.1 * f;
    // (ng-1) [2/R - (ng-1) t / (ng R^2)] = 1/f  <=>  R^2 - 2 (ng-1) f R + (ng-1)^2 f t / ng = 0
    const double p = (ng - 1.0) * f;
    const double disc = p * p - (ng - 1.0) * (ng - 1.0) * f * d->t / ng;
    if (!(disc >= 0.0)) return fail(c, PBR_ERR_ARG, "lens thickness admits no real radius");
    d->R = p + std::sqrt(disc);
    d->a = f / (2.0 * o.f_number);
    d->clear = o.clear_radius > 0.0 ? o.clear_radius : 1.5 * d->a;
    // reduced-angle system matrix [[A, B], [C, D]] of surface 1, glass, surface 2
    const double na = d->n_inf;
    const double ph1 = (ng - na) / d->R, ph2 = (na - ng) / (-d->R), tau = d->t / ng;
    const double A = 1.0 - tau * ph1, B = tau, C = -(ph1 + ph2 - tau * ph1 * ph2), D = 1.0 - tau * ph2;
    const double so = (o.z_front_vertex - o.z_focus) / na;   // reduced object distance
    const double si = -(A * so + B) / (C * so + D);          // reduced image distance
    const double z_img = o.z_front_vertex + d->t + si * na;
    d->M = A + si * C;
    d->z_sensor = std::isnan(s.z_sensor) ? z_img : s.z_sensor;
    if (s.sigma_px > 0.0) {
        d->sigma_px = s.sigma_px;
    } else {
        // eq. 8: d_tau = 2.44 (pi) f# (M + 1) lambda, sigma = d_tau / 4 (1/e^2 diameter)
        double dt = 2.44 * o.f_number * (std::fabs(d->M) + 1.0) * s.wavelength;
        if (s.dtau_with_pi) dt *= 3.14159265358979323846;
        d->sigma_px = dt / 4.0 / s.pitch;
    }
    d->rfp = (int)std::ceil(3.0 * d->sigma_px);
    if (d->rfp < 1) d->rfp = 1;
    if (d->rfp > pbr::kMaxFootprint)
        return fail(c, PBR_ERR_ARG, "spot sigma %.3g px needs a window wider than %d px", d->sigma_px,
                    2 * pbr::kMaxFootprint + 1);
    return PBR_OK;
}

int max_steps_for(const pbr_ctx *c, double ds)
{
    double d2 = 0.0;
    const int n3[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
        const double e = (double)(n3[a] - 1) * c->spacing[a];
        d2 += e * e;
    }
    const double m = 4.0 * std::ceil(std::sqrt(d2) / ds) + 64.0;
    return m > 67108864.0 ? 67108864 : (int)m;  // the step count is kept in 27 bits
}

// Launch parameters shared by the trace and the calibration (sources and rays left empty).
void fill_params(const pbr_ctx *ctx, const Derived &d, double ds, TraceParams *out)
{
    TraceParams &P = *out;
    std::memset(&P, 0, sizeof P);
    P.cells = ctx->cells;
    P.brick_fp64 = ctx->brick_fp64;
    P.nbx = ctx->layout.nbx; P.nby = ctx->layout.nby; P.nbz = ctx->layout.nbz;
    P.nx = ctx->nx; P.ny = ctx->ny; P.nz = ctx->nz;
    P.max_steps = max_steps_for(ctx, ds);
    const int n3[3] = {ctx->nx, ctx->ny, ctx->nz};
    P.h = ds / d.n_inf;
    for (int a = 0; a < 3; ++a) {
        P.origin[a] = ctx->origin[a];
        P.spacing[a] = ctx->spacing[a];
        P.lo[a] = ctx->origin[a];
        P.hi[a] = ctx->origin[a] + (double)(n3[a] - 1) * ctx->spacing[a];
        P.step_cell[a] = P.h / ctx->spacing[a];
    }
    // FP32 step constants (see TraceParams): each a float operation on float values, so that a
    // partial step of fraction 1 forms the same bits on the device
    float tlim = 3.0e38f;
    for (int a = 0; a < 3; ++a) {
        P.g32[a] = (float)P.step_cell[a];
        P.gh32[a] = 0.5f * P.g32[a];
        const double k = std::ceil(1.05 * (double)P.g32[a] + 4.0e-3);
        P.kin[a] = k < 1.0 ? 1 : (k > 1.0e6 ? 1000000 : (int)k);
        const float t = ((float)P.kin[a] - 4.0e-3f) / P.g32[a];
        tlim = t < tlim ? t : tlim;
    }
    P.h32 = (float)P.h;
    P.h4_32 = 0.25f * P.h32;
    P.h2_32 = 0.5f * P.h32;
    P.h6_32 = P.h32 * (1.0f / 6.0f);
    P.tlim32 = tlim;
    P.n_inf = d.n_inf;
    P.z_lens = ctx->has_chain ? ctx->chain.aim_z : ctx->optics.z_front_vertex;
    P.a = d.a; P.R = d.R; P.t = d.t; P.clear = d.clear; P.n_glass = ctx->optics.n_glass;
    P.z_sensor = d.z_sensor;
    P.accum = ctx->accum;
    P.W = ctx->sensor.width; P.H = ctx->sensor.height;
    P.pitch = ctx->sensor.pitch;
    P.sigma_px = d.sigma_px;
    P.rfp = d.rfp;
    P.node_layout = ctx->layout.nodes;
    P.rec = ctx->rec;
    P.rec_first = ctx->rec_first;
    P.rec_stride = ctx->rec_stride;
    P.rec_max = ctx->rec_max;
    P.counters = ctx->counters;
    P.chain = ctx->has_chain ? (const pbr_optical_chain *)((const char *)ctx->counters + pbr::kChainOffset) : nullptr;
}

int field_fingerprint(pbr_ctx *ctx, uint64_t *out)
{
    if (!ctx->has_field) return fail(ctx, PBR_ERR_STATE, "no field set");
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    // the counter block's spare slot after the queue holds the sum; only the bytes the field
    // preparation writes (not the alignment padding of the caller's workspace)
    unsigned long long *slot = ctx->counters + pbr::CNT_QUEUE + 1;
    const size_t bytes = ctx->layout.nodes ? (size_t)ctx->nx * (size_t)ctx->ny * (size_t)ctx->nz * 16
                                           : (size_t)(ctx->nx - 1) * (size_t)(ctx->ny - 1) * (size_t)(ctx->nz - 1) *
                                                 pbr::kCellFloat4 * 16;
    int e = pbr::launch_field_checksum(ctx->cells, bytes, slot, ctx->stream);
    unsigned long long h = 0;
    if (!e) e = (int)hipMemcpyAsync(&h, slot, 8, hipMemcpyDeviceToHost, ctx->stream);
    if (!e) e = (int)hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(ctx, e, "field checksum");
    *out = (uint64_t)h;
    return PBR_OK;
}

uint64_t next_uid()
{
    static std::atomic<uint64_t> n{0};
    return ++n;
}

}  // namespace host
}  // namespace pbr

using namespace pbr::host;

#define PBR_GUARD_BEGIN try {
#define PBR_GUARD_END                                                        \
    }                                                                        \
    catch (...) { return fail(ctx, PBR_ERR_HIP, "internal error (exception)"); }

extern "C" {

int pbr_create(pbr_ctx **out, int device, void *hip_stream)
{
    pbr_ctx *ctx = nullptr;
    PBR_GUARD_BEGIN
    if (!out) return fail(nullptr, PBR_ERR_ARG, "out is null");
    *out = nullptr;
    if (device == -1) {
        ctx = new (std::nothrow) pbr_ctx();
        if (!ctx) return fail(nullptr, PBR_ERR_HIP, "out of host memory");
        ctx->device = -1;
        ctx->uid = next_uid();
        *out = ctx;
        return PBR_OK;
    }
    int n = 0;
    int e = (int)hipGetDeviceCount(&n);
    if (e) return fail(nullptr, PBR_ERR_HIP, "hipGetDeviceCount: %s", hipGetErrorString((hipError_t)e));
    if (device < 0 || device >= n) return fail(nullptr, PBR_ERR_ARG, "device %d out of range (%d devices)", device, n);
    DeviceGuard g(device);
    if (!g.ok) return fail(nullptr, PBR_ERR_HIP, "hipSetDevice(%d) failed", device);
    ctx = new (std::nothrow) pbr_ctx();
    if (!ctx) return fail(nullptr, PBR_ERR_HIP, "out of host memory");
    ctx->device = device;
    ctx->uid = next_uid();
    ctx->stream = (hipStream_t)hip_stream;
    void *p = nullptr;
    e = (int)hipMalloc(&p, 4096);
    if (e) { delete ctx; return fail(nullptr, PBR_ERR_HIP, "hipMalloc(counters): %s", hipGetErrorString((hipError_t)e)); }
    ctx->counters = (unsigned long long *)p;
    if ((e = (int)hipEventCreate(&ctx->ev0)) || (e = (int)hipEventCreate(&ctx->ev1))) {
        (void)hipFree(p);
        delete ctx;
        return fail(nullptr, PBR_ERR_HIP, "hipEventCreate: %s", hipGetErrorString((hipError_t)e));
    }
    e = pbr::launch_clear_u64(ctx->counters, 4096 / 8, ctx->stream);
    if (e) { int r = hip_fail(nullptr, e, "clear counters"); (void)hipFree(p); delete ctx; return r; }
    // address of this device's static ray-state array (pbr_emit_and_trace_noalloc); a failed
    // lookup is reported by that call only
    (void)noalloc_scratch_init(device);
    *out = ctx;
    return PBR_OK;
    }
    catch (...) { delete ctx; return fail(nullptr, PBR_ERR_HIP, "internal error (exception)"); }
}

void pbr_destroy(pbr_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->device < 0) { delete ctx; return; }
    try {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        if (ctx->counters) (void)hipFree(ctx->counters);
        if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
        if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
        for (hipEvent_t ev : ctx->box_ev) (void)hipEventDestroy(ev);
    } catch (...) {
    }
    delete ctx;
}

const char *pbr_last_error(const pbr_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int pbr_set_stream(pbr_ctx *ctx, void *hip_stream)
{
    if (!ctx) return PBR_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return PBR_OK;
}

int pbr_checked_build(void)
{
    return PBR_CHECKED;
}

size_t pbr_field_workspace_bytes(int nx, int ny, int nz)
{
    if (nx < 2 || ny < 2 || nz < 2) return 0;
    return pbr::field_layout(nx, ny, nz).total;
}

size_t pbr_trace_workspace_bytes(int64_t rays_per_chunk)
{
    if (rays_per_chunk < 256) rays_per_chunk = 256;
    return (size_t)rays_per_chunk * sizeof(pbr::RayState);
}

int pbr_set_trace_workspace(pbr_ctx *ctx, void *ws_dev, size_t ws_bytes)
{
    if (!ctx) return PBR_ERR_ARG;
    if (!ws_dev) return fail(ctx, PBR_ERR_ARG, "trace workspace is null");
    if (((uintptr_t)ws_dev & 15u) != 0) return fail(ctx, PBR_ERR_ARG, "trace workspace must be 16-byte aligned");
    if (ws_bytes < pbr_trace_workspace_bytes(256))
        return fail(ctx, PBR_ERR_WORKSPACE, "trace workspace %zu bytes < %zu (256 rays)", ws_bytes,
                    pbr_trace_workspace_bytes(256));
    ctx->ray_ws = (pbr::RayState *)ws_dev;
    ctx->ray_chunk = (int64_t)(ws_bytes / sizeof(pbr::RayState));
    return PBR_OK;
}

namespace {
int set_field(pbr_ctx *ctx, const float *rho_dev, int nx, int ny, int nz, const double origin[3],
              const double spacing[3], double K, double rho_inf, void *ws_dev, size_t ws_bytes, bool nodes);
}  // namespace

int pbr_set_density_field(pbr_ctx *ctx, const float *rho_dev, int nx, int ny, int nz,
                          const double origin[3], const double spacing[3], double K,
                          double rho_inf, void *ws_dev, size_t ws_bytes)
{
    return set_field(ctx, rho_dev, nx, ny, nz, origin, spacing, K, rho_inf, ws_dev, ws_bytes, false);
}

int pbr_set_density_field_nodes(pbr_ctx *ctx, const float *rho_dev, int nx, int ny, int nz,
                                const double origin[3], const double spacing[3], double K,
                                double rho_inf, void *ws_dev, size_t ws_bytes)
{
    return set_field(ctx, rho_dev, nx, ny, nz, origin, spacing, K, rho_inf, ws_dev, ws_bytes, true);
}

size_t pbr_field_workspace_bytes_nodes(int nx, int ny, int nz)
{
    if (nx < 2 || ny < 2 || nz < 2) return 0;
    return pbr::field_layout(nx, ny, nz, true).total;
}

namespace {
int set_field(pbr_ctx *ctx, const float *rho_dev, int nx, int ny, int nz, const double origin[3],
              const double spacing[3], double K, double rho_inf, void *ws_dev, size_t ws_bytes, bool nodes)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    if (!rho_dev || !ws_dev || !origin || !spacing) return fail(ctx, PBR_ERR_ARG, "null pointer argument");
    if (nx < 2 || ny < 2 || nz < 2 || nx > 65535 || ny > 65535 || nz > 65535)
        return fail(ctx, PBR_ERR_ARG, "grid dimensions %d x %d x %d outside [2, 65535]", nx, ny, nz);
    if ((double)(nx - 1) * (ny - 1) * (nz - 1) > 2147483647.0)
        return fail(ctx, PBR_ERR_ARG, "grid has more than 2^31 - 1 cells");
    if (!finite3(origin) || !finite3(spacing)) return fail(ctx, PBR_ERR_ARG, "origin/spacing not finite");
    if (!(spacing[0] > 0 && spacing[1] > 0 && spacing[2] > 0)) return fail(ctx, PBR_ERR_ARG, "spacing must be > 0");
    if (!std::isfinite(K) || K < 0.0) return fail(ctx, PBR_ERR_ARG, "K must be finite and >= 0");
    if (!std::isfinite(rho_inf)) return fail(ctx, PBR_ERR_ARG, "rho_inf not finite");
    const size_t need = nodes ? pbr_field_workspace_bytes_nodes(nx, ny, nz) : pbr_field_workspace_bytes(nx, ny, nz);
    if (ws_bytes < need) return fail(ctx, PBR_ERR_WORKSPACE, "field workspace %zu bytes < %zu needed", ws_bytes, need);
    if (((uintptr_t)ws_dev & 15u) != 0) return fail(ctx, PBR_ERR_ARG, "field workspace must be 16-byte aligned");
    const pbr::FieldLayout L = pbr::field_layout(nx, ny, nz, nodes);
    char *base = (char *)ws_dev;
    if (ctx->device >= 0) {
        DeviceGuard g(ctx->device);
        if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
        // every density value must be finite: checked on the device before anything is prepared
        {
            unsigned long long *slot = ctx->counters + pbr::CNT_QUEUE + 2, bad = 0;
            int e = pbr::launch_check_finite(rho_dev, (int64_t)nx * ny * nz, slot, ctx->stream);
            if (!e) e = (int)hipMemcpyAsync(&bad, slot, 8, hipMemcpyDeviceToHost, ctx->stream);
            if (!e) e = (int)hipStreamSynchronize(ctx->stream);
            if (e) return hip_fail(ctx, e, "density check");
            if (bad) return fail(ctx, PBR_ERR_ARG, "the density grid holds non-finite values");
        }
        // brick max |grad n| and FP64 flags start at zero (fill kernel, no memset node)
        int e = pbr::launch_clear_u64((unsigned long long *)(base + L.gmax_off),
                                      (int64_t)((L.total - L.gmax_off) / 8), ctx->stream);
        if (e) return hip_fail(ctx, e, "clear brick tables");
        e = pbr::launch_field_prep(rho_dev, (float4 *)(base + L.cells_off), (unsigned *)(base + L.gmax_off),
                                   nx, ny, nz, spacing, K, ctx->stream, nodes);
        if (e) return hip_fail(ctx, e, "field preparation launch");
    }
    ctx->layout = L;
    ctx->brick_gmax = (unsigned *)(base + L.gmax_off);
    ctx->brick_fp64 = (unsigned char *)(base + L.flags_off);
    ctx->n_fp64_bricks = 0;
    ctx->cells = (const float4 *)(base + L.cells_off);
    ctx->nx = nx; ctx->ny = ny; ctx->nz = nz;
    for (int a = 0; a < 3; ++a) { ctx->origin[a] = origin[a]; ctx->spacing[a] = spacing[a]; }
    ctx->K = K;
    ctx->rho_inf = rho_inf;
    ctx->has_field = true;
    ++ctx->scene_version;
    ++ctx->param_version;
    return PBR_OK;
    PBR_GUARD_END
}
}  // namespace

int pbr_set_optics(pbr_ctx *ctx, const pbr_optics *o)
{
    if (!ctx) return PBR_ERR_ARG;
    if (!o) return fail(ctx, PBR_ERR_ARG, "optics is null");
    const double v[7] = {o->z_front_vertex, o->focal_length, o->f_number, o->thickness, o->n_glass,
                         o->clear_radius, o->z_focus};
    for (double x : v)
        if (!std::isfinite(x)) return fail(ctx, PBR_ERR_ARG, "optics values must be finite");
    if (!(o->focal_length > 0.0)) return fail(ctx, PBR_ERR_ARG, "focal_length must be > 0");
    if (!(o->f_number > 0.0)) return fail(ctx, PBR_ERR_ARG, "f_number must be > 0");
    if (!(o->n_glass > 1.0)) return fail(ctx, PBR_ERR_ARG, "n_glass must be > 1");
    const double t = o->thickness > 0.0 ? o->thickness : 0.1 * o->focal_length;
    if (t > o->n_glass * o->focal_length) return fail(ctx, PBR_ERR_ARG, "thickness > n_glass * focal_length");
    const double a = o->focal_length / (2.0 * o->f_number);
    if (o->clear_radius > 0.0 && o->clear_radius < a) return fail(ctx, PBR_ERR_ARG, "clear radius below aperture radius");
    ctx->optics = *o;
    ctx->has_optics = true;
    ++ctx->scene_version;
    ++ctx->param_version;
    return PBR_OK;
}

int pbr_set_sensor(pbr_ctx *ctx, const pbr_sensor *s, uint64_t *accum_dev)
{
    if (!ctx) return PBR_ERR_ARG;
    if (!s || !accum_dev) return fail(ctx, PBR_ERR_ARG, "null pointer argument");
    if (s->width < 1 || s->height < 1 || s->width > 16384 || s->height > 16384)
        return fail(ctx, PBR_ERR_ARG, "sensor %d x %d outside [1, 16384]", s->width, s->height);
    if (!(s->pitch > 0.0) || !std::isfinite(s->pitch)) return fail(ctx, PBR_ERR_ARG, "pitch must be finite and > 0");
    if (!std::isnan(s->z_sensor) && !std::isfinite(s->z_sensor)) return fail(ctx, PBR_ERR_ARG, "z_sensor must be finite or NaN");
    if (!(s->wavelength > 0.0) || !std::isfinite(s->wavelength)) return fail(ctx, PBR_ERR_ARG, "wavelength must be > 0");
    if (!std::isfinite(s->sigma_px)) return fail(ctx, PBR_ERR_ARG, "sigma_px not finite");
    if (((uintptr_t)accum_dev & 7u) != 0) return fail(ctx, PBR_ERR_ARG, "accumulator must be 8-byte aligned");
    ctx->sensor = *s;
    ctx->accum = (unsigned long long *)accum_dev;
    ctx->accum_rays = 0.0;  // unknown contents: the caller clears with PBR_CLEAR_FIRST
    ctx->has_sensor = true;
    ++ctx->scene_version;
    ++ctx->param_version;
    return PBR_OK;
}

int pbr_get_derived(pbr_ctx *ctx, pbr_derived *out)
{
    if (!ctx) return PBR_ERR_ARG;
    if (!out) return fail(ctx, PBR_ERR_ARG, "out is null");
    Derived d;
    const int r = derive(ctx, &d);
    if (r) return r;
    out->n_inf = d.n_inf;
    out->lens_radius = d.R;
    out->thickness = d.t;
    out->aperture_radius = d.a;
    out->clear_radius = d.clear;
    out->z_sensor = d.z_sensor;
    out->magnification = d.M;
    out->sigma_px = d.sigma_px;
    out->footprint_r = d.rfp;
    out->max_steps = ctx->last_max_steps;
    return PBR_OK;
}

int pbr_set_exit_recording(pbr_ctx *ctx, int64_t first, int64_t stride, int64_t max_records,
                           pbr_ray_exit *buf_dev)
{
    if (!ctx) return PBR_ERR_ARG;
    if (first < 0 || stride < 1 || max_records < 0) return fail(ctx, PBR_ERR_ARG, "bad recording range");
    if (max_records > 0 && !buf_dev) return fail(ctx, PBR_ERR_ARG, "record buffer is null");
    if (((uintptr_t)buf_dev & 7u) != 0) return fail(ctx, PBR_ERR_ARG, "record buffer must be 8-byte aligned");
    ctx->rec = buf_dev;
    ctx->rec_first = first;
    ctx->rec_stride = stride;
    ctx->rec_max = max_records;
    ++ctx->param_version;
    return PBR_OK;
}

int pbr_set_source_sums(pbr_ctx *ctx, pbr_source_sum *sums_dev, int64_t capacity)
{
    if (!ctx) return PBR_ERR_ARG;
    if (capacity < 0) return fail(ctx, PBR_ERR_ARG, "capacity < 0");
    if (capacity > 0 && !sums_dev) return fail(ctx, PBR_ERR_ARG, "sums array is null");
    if (((uintptr_t)sums_dev & 7u) != 0) return fail(ctx, PBR_ERR_ARG, "sums array must be 8-byte aligned");
    ctx->src_sums = capacity > 0 ? sums_dev : nullptr;
    ctx->src_sums_cap = capacity;
    return PBR_OK;
}

int pbr_set_source_order(pbr_ctx *ctx, const int64_t *order_dev, int64_t n_src)
{
    if (!ctx) return PBR_ERR_ARG;
    if (n_src < 0) return fail(ctx, PBR_ERR_ARG, "n_src < 0");
    if (n_src > 0 && !order_dev) return fail(ctx, PBR_ERR_ARG, "order array is null");
    if (((uintptr_t)order_dev & 7u) != 0) return fail(ctx, PBR_ERR_ARG, "order array must be 8-byte aligned");
    ctx->src_order = n_src > 0 ? order_dev : nullptr;
    ctx->src_order_n = n_src;
    return PBR_OK;
}

size_t pbr_source_order_morton_workspace_bytes(int64_t n_src) { return pbr::morton_order_scratch_bytes(n_src); }

int pbr_source_order_morton(pbr_ctx *ctx, const float *src_dev, int64_t n_src, int64_t *order_dev, void *ws_dev,
                            size_t ws_bytes)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    if (n_src < 0 || n_src > 2147483647) return fail(ctx, PBR_ERR_ARG, "n_src must lie in [0, 2^31 - 1]");
    if (n_src > 0 && (!src_dev || !order_dev)) return fail(ctx, PBR_ERR_ARG, "null source or order array");
    if (((uintptr_t)src_dev & 15u) != 0 || ((uintptr_t)order_dev & 7u) != 0)
        return fail(ctx, PBR_ERR_ARG, "misaligned source or order array");
    if (!ctx->has_field) return fail(ctx, PBR_ERR_STATE, "no field set");
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    const size_t need = pbr::morton_order_scratch_bytes(n_src);
    if (!ws_dev || ws_bytes < need)
        return fail(ctx, PBR_ERR_WORKSPACE, "order workspace of %zu bytes < %zu", ws_bytes, need);
    if (((uintptr_t)ws_dev & 255u) != 0) return fail(ctx, PBR_ERR_ARG, "order workspace must be 256-byte aligned");
    if (n_src == 0) return PBR_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    const int n3[3] = {ctx->nx, ctx->ny, ctx->nz};
    double ext[3];
    for (int a = 0; a < 3; ++a) ext[a] = (double)(n3[a] - 1) * ctx->spacing[a];
    const int e = pbr::launch_morton_order((const float4 *)src_dev, n_src, ctx->origin, ext, order_dev, ws_dev,
                                           ctx->stream);
    if (e) return hip_fail(ctx, e, "source order");
    return PBR_OK;
    PBR_GUARD_END
}

int pbr_emit_and_trace(pbr_ctx *ctx, const float *src_dev, int64_t n_src, int32_t rays_per_src,
                       uint64_t seed, double ds, uint32_t flags, pbr_stats *stats)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    return emit_and_trace_impl(ctx, src_dev, n_src, rays_per_src, seed, ds, flags, stats, false, nullptr, 0);
    PBR_GUARD_END
}

}  // extern "C"

namespace pbr {
namespace host {

int emit_and_trace_impl(pbr_ctx *ctx, const float *src_dev, int64_t n_src, int32_t rays_per_src, uint64_t seed,
                        double ds, uint32_t flags, pbr_stats *stats, bool noalloc, RayState *static_ws,
                        int64_t static_chunk)
{
    Derived d;
    int r = derive(ctx, &d);
    if (r) return r;
    if (n_src < 0) return fail(ctx, PBR_ERR_ARG, "n_src < 0");
    if (n_src > 0 && !src_dev) return fail(ctx, PBR_ERR_ARG, "source array is null");
    if (((uintptr_t)src_dev & 15u) != 0) return fail(ctx, PBR_ERR_ARG, "source array must be 16-byte aligned");
    if (rays_per_src < 1) return fail(ctx, PBR_ERR_ARG, "rays_per_src must be >= 1");
    if (!(ds > 0.0) || !std::isfinite(ds)) return fail(ctx, PBR_ERR_ARG, "ds must be finite and > 0");
    if (n_src > (int64_t)1 << 31) return fail(ctx, PBR_ERR_ARG, "n_src above 2^31");
    const double zmax = ctx->origin[2] + (double)(ctx->nz - 1) * ctx->spacing[2];
    if (ctx->has_chain) {
        if (!(ctx->chain.aim_z > zmax))
            return fail(ctx, PBR_ERR_ARG, "the chain's emission target must lie beyond the density box (z > %.6g)",
                        zmax);
    } else {
        if (!(ctx->optics.z_front_vertex > zmax))
            return fail(ctx, PBR_ERR_ARG, "lens front vertex must lie beyond the density box (z > %.6g)", zmax);
        if (!(d.z_sensor > ctx->optics.z_front_vertex + d.t))
            return fail(ctx, PBR_ERR_ARG, "sensor plane must lie behind the lens");
    }
    if (flags & ~(uint32_t)(PBR_CLEAR_FIRST | PBR_RECORD_EXITS | PBR_PREC_FP64_ALL | PBR_PREC_SHOCK_FP64 |
                            PBR_SURROGATE | PBR_LANE_REFILL | PBR_SOURCE_SUMS | PBR_MIE | PBR_SOURCE_ORDER))
        return fail(ctx, PBR_ERR_ARG, "unknown flag bits 0x%x", flags);
    if ((flags & PBR_MIE) && !ctx->mie) return fail(ctx, PBR_ERR_STATE, "no Mie table set (pbr_set_mie)");
    if (ctx->layout.nodes && (flags & PBR_LANE_REFILL))
        return fail(ctx, PBR_ERR_STATE, "lane refill needs the per-cell field (pbr_set_density_field)");
    if (flags & PBR_SOURCE_SUMS) {
        if (!ctx->src_sums) return fail(ctx, PBR_ERR_STATE, "no per-source sums set (pbr_set_source_sums)");
        if (n_src > ctx->src_sums_cap)
            return fail(ctx, PBR_ERR_WORKSPACE, "per-source sums hold %lld sources, the call has %lld",
                        (long long)ctx->src_sums_cap, (long long)n_src);
        if (rays_per_src > (1 << 25))
            return fail(ctx, PBR_ERR_ARG, "per-source sums need rays_per_src <= 2^25");
    }
    pbr::RayState *ray_ws = noalloc ? static_ws : ctx->ray_ws;
    const int64_t ray_chunk = noalloc ? static_chunk : ctx->ray_chunk;
    pbr::ChunkHook hook{nullptr, nullptr};
    if ((flags & PBR_SOURCE_ORDER) && n_src > 0) {
        if (!ctx->src_order) return fail(ctx, PBR_ERR_STATE, "no source order set (pbr_set_source_order)");
        if (ctx->src_order_n != n_src)
            return fail(ctx, PBR_ERR_ARG, "source order is for %lld sources, the call has %lld",
                        (long long)ctx->src_order_n, (long long)n_src);
    }
    if (flags & PBR_SURROGATE) {
        if ((r = surrogate_hook(ctx, ds, ray_chunk, &hook))) return r;
    }
    if (!noalloc && !ray_ws) return fail(ctx, PBR_ERR_STATE, "no trace workspace set (pbr_set_trace_workspace)");
    if ((flags & PBR_RECORD_EXITS) && ctx->rec_max > 0 && !ctx->rec)
        return fail(ctx, PBR_ERR_STATE, "no exit recording buffer set");
    const double n_rays_d = (double)n_src * (double)rays_per_src;
    const double before = (flags & PBR_CLEAR_FIRST) ? 0.0 : ctx->accum_rays;
    // each ray adds at most 2^32 to a pixel (weight <= 1): the sum stays below 2^64
    if (before + n_rays_d > 4294967295.0)
        return fail(ctx, PBR_ERR_OVERFLOW, "more than 2^32 - 1 rays per accumulation; clear the sensor");

    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    if (!ray_ws) return fail(ctx, PBR_ERR_STATE, "no static ray-state array on device %d", ctx->device);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    int e;
    if (flags & PBR_CLEAR_FIRST) {
        e = pbr::launch_clear_u64(ctx->accum, (int64_t)ctx->sensor.width * ctx->sensor.height, ctx->stream);
        if (e) return hip_fail(ctx, e, "clear sensor");
    }
    e = pbr::launch_clear_u64(ctx->counters, pbr::CNT_SLOTS, ctx->stream);
    if (e) return hip_fail(ctx, e, "clear counters");

    pbr::TraceParams P;
    fill_params(ctx, d, ds, &P);
    P.src = (const float4 *)src_dev;
    P.n_src = n_src;
    P.rays_per_src = rays_per_src;
    P.n_rays = n_src * (int64_t)rays_per_src;
    P.seed = seed;
    P.record = (flags & PBR_RECORD_EXITS) && ctx->rec_max > 0 ? 1 : 0;
    P.src_sums = (flags & PBR_SOURCE_SUMS) ? ctx->src_sums : nullptr;
    P.order = (flags & PBR_SOURCE_ORDER) && n_src > 0 ? ctx->src_order : nullptr;
    if (flags & PBR_MIE) {
        P.mie = ctx->mie;
        P.mie_n = PBR_MIE_TABLE_SIZE;
        for (int a = 0; a < 3; ++a) P.laser[a] = ctx->laser[a];
    }
    ctx->last_max_steps = P.max_steps;

    const int prec = (flags & PBR_PREC_FP64_ALL) ? pbr::PREC_FP64
                     : ((flags & PBR_PREC_SHOCK_FP64) && ctx->n_fp64_bricks > 0) ? pbr::PREC_MIXED
                     : pbr::PREC_FP32;
    const int64_t n_chunks = (P.n_rays + ray_chunk - 1) / ray_chunk;
    // per-launch timing events (created on demand, so not in the allocation-free variant)
    const bool launch_ev = stats && !noalloc;
    if (stats) {
        while (launch_ev && (int64_t)ctx->box_ev.size() < 2 * n_chunks) {
            hipEvent_t ev;
            if ((e = (int)hipEventCreate(&ev))) return hip_fail(ctx, e, "hipEventCreate");
            ctx->box_ev.push_back(ev);
        }
        if ((e = (int)hipEventRecord(ctx->ev0, ctx->stream))) return hip_fail(ctx, e, "hipEventRecord");
    }
    for (int64_t k = 0; k < n_chunks; ++k) {
        const int64_t first = k * ray_chunk;
        const int64_t n = P.n_rays - first < ray_chunk ? P.n_rays - first : ray_chunk;
        e = pbr::launch_trace_chunk(P, ray_ws, first, n, prec, ctx->stream,
                                    launch_ev ? ctx->box_ev[2 * k] : nullptr, launch_ev ? ctx->box_ev[2 * k + 1] : nullptr,
                                    hook.run ? &hook : nullptr, true, (flags & PBR_LANE_REFILL) != 0);
        if (e) return hip_fail(ctx, e, "trace launch");
    }
    if (stats && (e = (int)hipEventRecord(ctx->ev1, ctx->stream))) return hip_fail(ctx, e, "hipEventRecord");
    ctx->accum_rays = before + n_rays_d;

    if (stats) {
        unsigned long long h[pbr::CNT_SLOTS];
        e = (int)hipMemcpyAsync(h, ctx->counters, sizeof h, hipMemcpyDeviceToHost, ctx->stream);
        if (e) return hip_fail(ctx, e, "copy counters");
        e = (int)hipStreamSynchronize(ctx->stream);
        if (e) return hip_fail(ctx, e, "trace (stream synchronise)");
        float ms = 0.0f;
        e = (int)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        if (e) return hip_fail(ctx, e, "hipEventElapsedTime");
        std::memset(stats, 0, sizeof *stats);
        stats->rays = (uint64_t)P.n_rays;
        for (int k = 0; k < PBR_NUM_STATUS; ++k) stats->status[k] = h[pbr::CNT_STATUS + k];
        stats->entered_volume = h[pbr::CNT_ENTERED];
        stats->rkn_steps = h[pbr::CNT_STEPS];
        stats->rkn_steps_fp64 = prec == pbr::PREC_FP64 ? h[pbr::CNT_STEPS] : h[pbr::CNT_STEPS64];
        stats->surrogate_rays = h[pbr::CNT_SURR];
        stats->trace_ms = (double)ms;
        double box = 0.0;
        for (int64_t k = 0; launch_ev && k < n_chunks; ++k) {
            float b = 0.0f;
            e = (int)hipEventElapsedTime(&b, ctx->box_ev[2 * k], ctx->box_ev[2 * k + 1]);
            if (e) return hip_fail(ctx, e, "hipEventElapsedTime");
            box += (double)b;
        }
        stats->box_ms = box;
        stats->box_launches = (uint64_t)n_chunks;
    }
#if PBR_CHECKED
    unsigned long long bad = 0;
    e = (int)hipMemcpyAsync(&bad, ctx->counters + pbr::CNT_BAD_ACCESS, sizeof bad, hipMemcpyDeviceToHost, ctx->stream);
    if (!e) e = (int)hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(ctx, e, "read the checked-access counter");
    if (bad)
        return fail(ctx, PBR_ERR_BOUNDS, "checked build: %llu device accesses outside their buffers (clamped or skipped)",
                    bad);
#endif
    return PBR_OK;
}

}  // namespace host
}  // namespace pbr

extern "C" {

int pbr_calibrate_precision(pbr_ctx *ctx, double tol_px, double steep_frac, int32_t rays_per_brick,
                            uint64_t seed, double ds, pbr_precision_report *out)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    Derived d;
    int r = derive(ctx, &d);
    if (r) return r;
    if (ctx->has_chain) return fail(ctx, PBR_ERR_STATE, "precision calibration needs the singlet (an optical chain is set)");
    if (!(tol_px >= 0.0) || !std::isfinite(tol_px)) return fail(ctx, PBR_ERR_ARG, "tol_px must be finite and >= 0");
    if (!(steep_frac >= 0.0 && steep_frac <= 1.0)) return fail(ctx, PBR_ERR_ARG, "steep_frac must lie in [0, 1]");
    if (rays_per_brick < 1 || rays_per_brick > 256) return fail(ctx, PBR_ERR_ARG, "rays_per_brick must lie in [1, 256]");
    if (!(ds > 0.0) || !std::isfinite(ds)) return fail(ctx, PBR_ERR_ARG, "ds must be finite and > 0");
    if (!ctx->ray_ws) return fail(ctx, PBR_ERR_STATE, "no trace workspace set (used as calibration scratch)");
    const int64_t nb = ctx->layout.n_bricks;
    if ((size_t)nb * 8 > (size_t)ctx->ray_chunk * sizeof(pbr::RayState))
        return fail(ctx, PBR_ERR_WORKSPACE, "trace workspace too small for %lld calibration bricks", (long long)nb);
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    std::vector<unsigned> gmax((size_t)nb);
    int e = (int)hipMemcpyAsync(gmax.data(), ctx->brick_gmax, (size_t)nb * 4, hipMemcpyDeviceToHost, ctx->stream);
    if (!e) e = (int)hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(ctx, e, "read brick steepness");
    float gtop = 0.0f;
    for (unsigned v : gmax) { float f; std::memcpy(&f, &v, 4); gtop = f > gtop ? f : gtop; }
    const float thr = (float)(steep_frac * (double)gtop);
    std::vector<int> steep;
    for (int64_t b = 0; b < nb; ++b) {
        float f;
        std::memcpy(&f, &gmax[(size_t)b], 4);
        if (f > 0.0f && f >= thr) steep.push_back((int)b);
    }
    const int ns = (int)steep.size();
    double smax = 0.0;
    for (int a = 0; a < 3; ++a) smax = ctx->spacing[a] > smax ? ctx->spacing[a] : smax;
    int n_steps = (int)std::ceil((double)pbr::kBrick * smax * 1.7320508075688772 / ds) + 1;
    n_steps = n_steps > 512 ? 512 : n_steps;
    std::vector<float> err((size_t)ns, 0.0f);
    if (ns > 0) {
        int *dev_list = (int *)ctx->ray_ws;
        float *dev_err = (float *)((char *)ctx->ray_ws + (size_t)ns * 4);
        e = (int)hipMemcpyAsync(dev_list, steep.data(), (size_t)ns * 4, hipMemcpyHostToDevice, ctx->stream);
        if (e) return hip_fail(ctx, e, "upload brick list");
        pbr::TraceParams P;
        fill_params(ctx, d, ds, &P);
#if PBR_CHECKED
        if ((e = pbr::launch_clear_u64(ctx->counters + pbr::CNT_BAD_ACCESS, 1, ctx->stream)))
            return hip_fail(ctx, e, "clear the checked-access counter");
#endif
        e = pbr::launch_calibrate(P, dev_list, ns, rays_per_brick, n_steps, seed, ctx->optics.z_focus,
                                  std::fabs(d.M) / ctx->sensor.pitch, dev_err, ctx->stream);
        if (e) return hip_fail(ctx, e, "calibration launch");
        e = (int)hipMemcpyAsync(err.data(), dev_err, (size_t)ns * 4, hipMemcpyDeviceToHost, ctx->stream);
        if (!e) e = (int)hipStreamSynchronize(ctx->stream);
        if (e) return hip_fail(ctx, e, "calibration");
#if PBR_CHECKED
        unsigned long long bad = 0;
        e = (int)hipMemcpy(&bad, ctx->counters + pbr::CNT_BAD_ACCESS, sizeof bad, hipMemcpyDeviceToHost);
        if (e) return hip_fail(ctx, e, "read the checked-access counter");
        if (bad)
            return fail(ctx, PBR_ERR_BOUNDS, "checked build: calibration made %llu device accesses outside their "
                        "buffers (clamped or skipped)", bad);
#endif
    }
    std::vector<unsigned char> flags((size_t)nb, 0);
    int64_t nf = 0;
    double emax = 0.0;
    for (int k = 0; k < ns; ++k) {
        emax = err[(size_t)k] > emax ? err[(size_t)k] : emax;
        if ((double)err[(size_t)k] > tol_px) { flags[(size_t)steep[(size_t)k]] = 1; ++nf; }
    }
    e = (int)hipMemcpyAsync(ctx->brick_fp64, flags.data(), (size_t)nb, hipMemcpyHostToDevice, ctx->stream);
    if (!e) e = (int)hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(ctx, e, "write brick flags");
    ctx->n_fp64_bricks = nf;
    if (out) {
        out->n_bricks = nb;
        out->n_steep = ns;
        out->n_fp64 = nf;
        out->grad_threshold = (double)thr;
        out->grad_max = (double)gtop;
        out->max_err_px = emax;
        out->tol_px = tol_px;
        out->steps_per_sample = n_steps;
        out->rays_per_brick = rays_per_brick;
    }
    return PBR_OK;
    PBR_GUARD_END
}

int pbr_brick_flags(pbr_ctx *ctx, uint8_t *inout_host, int64_t n_bricks, int write)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    if (!ctx->has_field) return fail(ctx, PBR_ERR_STATE, "no density field set");
    if (!inout_host || n_bricks != ctx->layout.n_bricks)
        return fail(ctx, PBR_ERR_ARG, "need a host array of %lld brick flags", (long long)ctx->layout.n_bricks);
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    int e;
    if (write) {
        int64_t nf = 0;
        for (int64_t b = 0; b < n_bricks; ++b) nf += inout_host[b] ? 1 : 0;
        e = (int)hipMemcpyAsync(ctx->brick_fp64, inout_host, (size_t)n_bricks, hipMemcpyHostToDevice, ctx->stream);
        if (!e) e = (int)hipStreamSynchronize(ctx->stream);
        if (e) return hip_fail(ctx, e, "write brick flags");
        ctx->n_fp64_bricks = nf;
    } else {
        e = (int)hipMemcpyAsync(inout_host, ctx->brick_fp64, (size_t)n_bricks, hipMemcpyDeviceToHost, ctx->stream);
        if (!e) e = (int)hipStreamSynchronize(ctx->stream);
        if (e) return hip_fail(ctx, e, "read brick flags");
    }
    return PBR_OK;
    PBR_GUARD_END
}

int pbr_read_image(pbr_ctx *ctx, int fmt, void *out_dev, double gain)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    if (!ctx->has_sensor) return fail(ctx, PBR_ERR_STATE, "no sensor set");
    if (!out_dev) return fail(ctx, PBR_ERR_ARG, "out is null");
    if (fmt != PBR_FMT_RAW_U64 && fmt != PBR_FMT_F32 && fmt != PBR_FMT_U16)
        return fail(ctx, PBR_ERR_ARG, "unknown image format %d", fmt);
    const size_t align = fmt == PBR_FMT_RAW_U64 ? 8 : fmt == PBR_FMT_F32 ? 4 : 2;
    if (((uintptr_t)out_dev % align) != 0) return fail(ctx, PBR_ERR_ARG, "output misaligned");
    if (!std::isfinite(gain)) return fail(ctx, PBR_ERR_ARG, "gain not finite");
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    const int e = pbr::launch_readout(ctx->accum, (int64_t)ctx->sensor.width * ctx->sensor.height, fmt,
                                      out_dev, gain, ctx->counters, ctx->stream);
    if (e) return hip_fail(ctx, e, "readout launch");
    return PBR_OK;
    PBR_GUARD_END
}

namespace {
int check_grid(pbr_ctx *ctx, const pbr_map_grid *g)
{
    if (!g) return fail(ctx, PBR_ERR_ARG, "grid is null");
    if (g->nx < 1 || g->ny < 1 || g->nx > 4096 || g->ny > 4096)
        return fail(ctx, PBR_ERR_ARG, "grid nodes must be 1 .. 4096 per axis");
    if (!(g->dx > 0.0) || !(g->dy > 0.0) || !std::isfinite(g->dx) || !std::isfinite(g->dy) ||
        !std::isfinite(g->x0) || !std::isfinite(g->y0) || !std::isfinite(g->z_dots))
        return fail(ctx, PBR_ERR_ARG, "grid spacing must be finite and > 0, origin finite");
    return PBR_OK;
}
}  // namespace

size_t pbr_dot_map_workspace_bytes(int nx, int ny)
{
    if (nx < 1 || ny < 1 || nx > 4096 || ny > 4096) return 0;
    return (size_t)nx * (size_t)ny * 24u;
}

int pbr_dot_displacement_map(pbr_ctx *ctx, const pbr_source_sum *with_dev, const pbr_source_sum *without_dev,
                             const float *src_dev, int64_t n_src, const pbr_map_grid *grid, void *ws_dev,
                             size_t ws_bytes, float *map_dev)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    int r = check_grid(ctx, grid);
    if (r) return r;
    if (n_src < 0) return fail(ctx, PBR_ERR_ARG, "n_src < 0");
    if (n_src > 0 && (!with_dev || !without_dev || !src_dev))
        return fail(ctx, PBR_ERR_ARG, "sums or source array is null");
    if (!map_dev || !ws_dev) return fail(ctx, PBR_ERR_ARG, "map or workspace is null");
    if ((((uintptr_t)with_dev | (uintptr_t)without_dev | (uintptr_t)ws_dev) & 7u) != 0 ||
        ((uintptr_t)src_dev & 15u) != 0 || ((uintptr_t)map_dev & 3u) != 0)
        return fail(ctx, PBR_ERR_ARG, "misaligned array (sums and workspace 8, sources 16, map 4 bytes)");
    if (ws_bytes < pbr_dot_map_workspace_bytes(grid->nx, grid->ny))
        return fail(ctx, PBR_ERR_WORKSPACE, "map workspace needs %zu bytes",
                    pbr_dot_map_workspace_bytes(grid->nx, grid->ny));
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    const int e = pbr::launch_dot_map(with_dev, without_dev, (const float4 *)src_dev, n_src, *grid,
                                      (unsigned long long *)ws_dev, map_dev, ctx->stream);
    if (e) return hip_fail(ctx, e, "displacement map launch");
    return PBR_OK;
    PBR_GUARD_END
}

int pbr_bos_theory_map(pbr_ctx *ctx, const pbr_map_grid *grid, int32_t samples, float *map_dev)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    Derived d;
    int r = derive(ctx, &d);
    if (r) return r;
    if (ctx->has_chain) return fail(ctx, PBR_ERR_STATE, "the eq. 9 map needs the singlet's magnification (an optical chain is set)");
    if ((r = check_grid(ctx, grid))) return r;
    if (samples < 1 || samples > 65536) return fail(ctx, PBR_ERR_ARG, "samples must be 1 .. 65536");
    if (!map_dev || ((uintptr_t)map_dev & 3u) != 0) return fail(ctx, PBR_ERR_ARG, "map is null or misaligned");
    if (!(grid->z_dots < ctx->origin[2])) return fail(ctx, PBR_ERR_ARG, "dot plane must lie in front of the box");
    // paraxial magnification of the dot plane (system matrix of derive, object at z_dots)
    const pbr_optics &o = ctx->optics;
    const double na = d.n_inf, ng = o.n_glass;
    const double ph1 = (ng - na) / d.R, ph2 = (na - ng) / (-d.R), tau = d.t / ng;
    const double A = 1.0 - tau * ph1, B = tau, C = -(ph1 + ph2 - tau * ph1 * ph2), D = 1.0 - tau * ph2;
    const double so = (o.z_front_vertex - grid->z_dots) / na;
    const double si = -(A * so + B) / (C * so + D);
    const double M = A + si * C;
    const double zc = ctx->origin[2] + 0.5 * (double)(ctx->nz - 1) * ctx->spacing[2];
    const double scale = std::fabs(M) * (zc - grid->z_dots) / (d.n_inf * ctx->sensor.pitch);
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    pbr::TraceParams P;
    fill_params(ctx, d, 1e-4, &P);
    const int e = pbr::launch_bos_theory(P, *grid, scale, samples, map_dev, ctx->stream);
    if (e) return hip_fail(ctx, e, "theory map launch");
    return PBR_OK;
    PBR_GUARD_END
}

int pbr_displace_sources(pbr_ctx *ctx, const float *src_in_dev, float *src_out_dev, int64_t n_src,
                         const float *vel_dev, int nx, int ny, int nz, const double origin[3],
                         const double spacing[3], double dt, int32_t substeps)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    if (n_src < 0) return fail(ctx, PBR_ERR_ARG, "n_src < 0");
    if (n_src > 0 && (!src_in_dev || !src_out_dev)) return fail(ctx, PBR_ERR_ARG, "source array is null");
    if ((((uintptr_t)src_in_dev | (uintptr_t)src_out_dev) & 15u) != 0)
        return fail(ctx, PBR_ERR_ARG, "source arrays must be 16-byte aligned");
    if (!vel_dev || ((uintptr_t)vel_dev & 3u) != 0) return fail(ctx, PBR_ERR_ARG, "velocity is null or misaligned");
    if (!origin || !spacing) return fail(ctx, PBR_ERR_ARG, "origin or spacing is null");
    if (nx < 2 || ny < 2 || nz < 2 || nx > 65535 || ny > 65535 || nz > 65535 ||
        (double)nx * ny * nz > 2147483647.0)
        return fail(ctx, PBR_ERR_ARG, "velocity grid must have 2 .. 65535 nodes per axis, at most 2^31 - 1 nodes");
    if (!finite3(origin) || !finite3(spacing) || !(spacing[0] > 0.0) || !(spacing[1] > 0.0) || !(spacing[2] > 0.0))
        return fail(ctx, PBR_ERR_ARG, "velocity grid origin must be finite, spacing finite and > 0");
    if (!std::isfinite(dt)) return fail(ctx, PBR_ERR_ARG, "dt must be finite");
    if (substeps < 1 || substeps > 4096) return fail(ctx, PBR_ERR_ARG, "substeps must be 1 .. 4096");
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    pbr::VelocityGrid vg;
    vg.vel = vel_dev;
    vg.nx = nx; vg.ny = ny; vg.nz = nz;
    for (int a = 0; a < 3; ++a) { vg.origin[a] = origin[a]; vg.spacing[a] = spacing[a]; }
    const int e = pbr::launch_displace((const float4 *)src_in_dev, (float4 *)src_out_dev, n_src, vg, dt, substeps,
                                       ctx->stream);
    if (e) return hip_fail(ctx, e, "displacement launch");
    return PBR_OK;
    PBR_GUARD_END
}

namespace {
int check_mie(pbr_ctx *ctx, const pbr_mie *m, double n_medium, double *x)
{
    if (!std::isfinite(m->diameter) || !(m->diameter > 0.0) || !std::isfinite(m->wavelength) ||
        !(m->wavelength > 0.0) || !std::isfinite(m->m_re) || !(m->m_re > 0.0) || !std::isfinite(m->m_im) ||
        m->m_im < 0.0 || !finite3(m->laser_dir))
        return fail(ctx, PBR_ERR_ARG, "Mie particle: diameter, wavelength, m_re > 0, m_im >= 0, finite direction");
    const double k2 = m->laser_dir[0] * m->laser_dir[0] + m->laser_dir[1] * m->laser_dir[1] +
                      m->laser_dir[2] * m->laser_dir[2];
    if (!(k2 > 0.0)) return fail(ctx, PBR_ERR_ARG, "laser direction is zero");
    if (!std::isfinite(n_medium) || !(n_medium > 0.0)) return fail(ctx, PBR_ERR_ARG, "medium index must be > 0");
    *x = 3.14159265358979323846 * m->diameter * n_medium / m->wavelength;
    if (*x > 20000.0) return fail(ctx, PBR_ERR_ARG, "size parameter %.6g above 20000", *x);
    return PBR_OK;
}
}  // namespace

int pbr_mie_table(const pbr_mie *mie, double n_medium, double *out_host, int32_t n)
{
    pbr_ctx *ctx = nullptr;
    PBR_GUARD_BEGIN
    if (!mie || !out_host) return fail(nullptr, PBR_ERR_ARG, "null argument");
    if (n < 2) return fail(nullptr, PBR_ERR_ARG, "table needs at least 2 angles");
    double x;
    int r = check_mie(nullptr, mie, n_medium, &x);
    if (r) return r;
    if (!mie_intensity_table(std::complex<double>(mie->m_re, mie->m_im), x, n, out_host))
        return fail(nullptr, PBR_ERR_ARG, "Mie intensity vanishes or overflows");
    return PBR_OK;
    PBR_GUARD_END
}

size_t pbr_mie_workspace_bytes(void) { return (size_t)PBR_MIE_TABLE_SIZE * sizeof(double); }

int pbr_set_mie(pbr_ctx *ctx, const pbr_mie *mie, void *table_dev, size_t ws_bytes)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    if (!mie) {
        ctx->mie = nullptr;
        return PBR_OK;
    }
    if (!ctx->has_field) return fail(ctx, PBR_ERR_STATE, "set the density field first (ambient index)");
    double x;
    int r = check_mie(ctx, mie, 1.0 + ctx->K * ctx->rho_inf, &x);
    if (r) return r;
    if (!table_dev || ((uintptr_t)table_dev & 7u) != 0) return fail(ctx, PBR_ERR_ARG, "table is null or misaligned");
    if (ws_bytes < pbr_mie_workspace_bytes())
        return fail(ctx, PBR_ERR_WORKSPACE, "Mie table needs %zu bytes", pbr_mie_workspace_bytes());
    std::vector<double> t(PBR_MIE_TABLE_SIZE);
    if (!mie_intensity_table(std::complex<double>(mie->m_re, mie->m_im), x, PBR_MIE_TABLE_SIZE, t.data()))
        return fail(ctx, PBR_ERR_ARG, "Mie intensity vanishes or overflows");
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    int e = (int)hipMemcpyAsync(table_dev, t.data(), pbr_mie_workspace_bytes(), hipMemcpyHostToDevice, ctx->stream);
    if (!e) e = (int)hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(ctx, e, "Mie table copy");
    const double k = std::sqrt(mie->laser_dir[0] * mie->laser_dir[0] + mie->laser_dir[1] * mie->laser_dir[1] +
                               mie->laser_dir[2] * mie->laser_dir[2]);
    for (int a = 0; a < 3; ++a) ctx->laser[a] = mie->laser_dir[a] / k;
    ctx->mie = (const double *)table_dev;
    return PBR_OK;
    PBR_GUARD_END
}

int pbr_set_optical_chain(pbr_ctx *ctx, const pbr_optical_chain *chain)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    if (!chain) {
        ctx->has_chain = false;
        ctx->scene_version++;
        ctx->param_version++;
        return PBR_OK;
    }
    if (chain->n_surfaces < 1 || chain->n_surfaces > PBR_MAX_SURFACES)
        return fail(ctx, PBR_ERR_ARG, "chain needs 1 .. %d surfaces", PBR_MAX_SURFACES);
    if (!std::isfinite(chain->aim_z) || !std::isfinite(chain->aim_radius) || !(chain->aim_radius > 0.0))
        return fail(ctx, PBR_ERR_ARG, "emission target: finite plane and radius > 0");
    for (int k = 0; k < chain->n_surfaces; ++k) {
        const pbr_surface &f = chain->s[k];
        if (f.type < PBR_SURF_REFRACT || f.type > PBR_SURF_LENSLETS)
            return fail(ctx, PBR_ERR_ARG, "surface %d: unknown type %d", k, f.type);
        if (!std::isfinite(f.z) || !std::isfinite(f.radius) || !std::isfinite(f.clear) || !(f.clear > 0.0) ||
            !std::isfinite(f.n_after) || !std::isfinite(f.pitch))
            return fail(ctx, PBR_ERR_ARG, "surface %d: finite z, radius, index, pitch and clear > 0", k);
        if (f.type == PBR_SURF_LENSLETS && (!(f.pitch > 0.0) || (f.radius != 0.0 && std::fabs(f.radius) < 0.5 * f.pitch)))
            return fail(ctx, PBR_ERR_ARG, "surface %d: lenslet pitch > 0 and |radius| >= pitch / 2", k);
    }
    if (ctx->device >= 0) {
        DeviceGuard g(ctx->device);
        if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
        int e = (int)hipMemcpyAsync((char *)ctx->counters + pbr::kChainOffset, chain, sizeof(pbr_optical_chain),
                                    hipMemcpyHostToDevice, ctx->stream);
        if (!e) e = (int)hipStreamSynchronize(ctx->stream);
        if (e) return hip_fail(ctx, e, "optical chain copy");
    }
    ctx->chain = *chain;
    ctx->has_chain = true;
    ctx->scene_version++;
    ctx->param_version++;
    return PBR_OK;
    PBR_GUARD_END
}

int pbr_read_ray_exits(pbr_ctx *ctx, pbr_ray_exit *out_host, int64_t first, int64_t count)
{
    if (!ctx) return PBR_ERR_ARG;
    PBR_GUARD_BEGIN
    if (!ctx->rec || ctx->rec_max == 0) return fail(ctx, PBR_ERR_STATE, "no exit recording set");
    if (first < 0 || count < 0 || first + count > ctx->rec_max) return fail(ctx, PBR_ERR_ARG, "record range outside the buffer");
    if (count > 0 && !out_host) return fail(ctx, PBR_ERR_ARG, "out is null");
    if (count == 0) return PBR_OK;
    if (ctx->device < 0) return fail(ctx, PBR_ERR_STATE, "host-only context: no device work");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, PBR_ERR_HIP, "hipSetDevice failed");
    int e = (int)hipMemcpyAsync(out_host, ctx->rec + first, (size_t)count * sizeof(pbr_ray_exit),
                                hipMemcpyDeviceToHost, ctx->stream);
    if (e) return hip_fail(ctx, e, "copy records");
    e = (int)hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(ctx, e, "records (stream synchronise)");
    return PBR_OK;
    PBR_GUARD_END
}

}  // extern "C"
