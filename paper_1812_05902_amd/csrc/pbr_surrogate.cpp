// Host side of the ray surrogate network (include/pbr.h): parameters and Adam state on the device,
// the training loop over rays the tracer integrates, the validation that fixes the fallback map,
// and the per-chunk hook that hands eligible rays to the network during a trace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mlp_internal.h"
#include "pbr_ctx.h"

using pbr::host::DeviceGuard;

struct pbr_surrogate {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int64_t rows_cap = 0;
    pbr::MlpDevice d{};
    pbr::MlpTrain tb{};
    float *x = nullptr, *y = nullptr, *t = nullptr, *loss = nullptr;
    int *step = nullptr;                 // training step counter read by the captured step
    hipStream_t train_stream = nullptr;  // non-blocking stream the training step is captured on
    hipStream_t copy_stream = nullptr;   // uploads of the next epoch's order while an epoch runs
    int *idx = nullptr;
    unsigned long long *count = nullptr;
    // trained state
    bool trained = false;
    uint64_t ctx_uid = 0, scene_version = 0;
    pbr::SurrogateSpec spec{};
    unsigned char *tile_ok_dev = nullptr;  // kMaxTiles^2 bytes
    // inference on whole trace chunks: features, outputs, row -> ray index, rays left to the tracer
    float *ix = nullptr, *iy = nullptr;
    unsigned char *ielig = nullptr;
    int *tlist = nullptr;
    int64_t chunk_cap = 0;
    std::vector<unsigned char> tile_ok;
    std::vector<float> tile_err;
    // what the trained state depends on (checked when a saved surrogate is loaded)
    double ds = 0.0;
    struct SceneKey {
        int32_t nx, ny, nz, node_layout;
        double origin[3], spacing[3], K, rho_inf, ds;
        uint64_t field_sum, optics_hash;
    } key{};
};

namespace {

thread_local std::string g_surr_create_err;

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 0xcbf29ce484222325ull)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t k = 0; k < n; ++k) h = (h ^ b[k]) * 0x100000001b3ull;
    return h;
}

// Host-side fingerprint of the optics, sensor and optical chain (field by field: no padding bytes).
uint64_t optics_hash(const pbr_ctx *c)
{
    uint64_t h = fnv1a(nullptr, 0);
    const pbr_optics &o = c->optics;
    const double od[7] = {o.z_front_vertex, o.focal_length, o.f_number, o.thickness, o.n_glass, o.clear_radius,
                          o.z_focus};
    h = fnv1a(od, sizeof od, h);
    const pbr_sensor &q = c->sensor;
    const int32_t si[3] = {q.width, q.height, q.dtau_with_pi};
    const double sd[4] = {q.pitch, q.z_sensor, q.wavelength, q.sigma_px};
    h = fnv1a(si, sizeof si, h);
    h = fnv1a(sd, sizeof sd, h);
    const int32_t chain = c->has_chain ? c->chain.n_surfaces : 0;
    h = fnv1a(&chain, sizeof chain, h);
    if (chain) {
        const double aim[2] = {c->chain.aim_z, c->chain.aim_radius};
        h = fnv1a(aim, sizeof aim, h);
        for (int k = 0; k < chain; ++k) {
            const pbr_surface &f = c->chain.s[k];
            const double fd[5] = {f.z, f.radius, f.clear, f.n_after, f.pitch};
            h = fnv1a(&f.type, sizeof f.type, h);
            h = fnv1a(fd, sizeof fd, h);
        }
    }
    return h;
}

// What a trained surrogate depends on: the stored field (geometry and a device checksum of its
// words), the optics and sensor it was validated through, and the step length.
int scene_key(pbr_ctx *ctx, double ds, pbr_surrogate::SceneKey *k)
{
    std::memset(k, 0, sizeof *k);
    k->nx = ctx->nx; k->ny = ctx->ny; k->nz = ctx->nz;
    k->node_layout = ctx->layout.nodes;
    for (int a = 0; a < 3; ++a) { k->origin[a] = ctx->origin[a]; k->spacing[a] = ctx->spacing[a]; }
    k->K = ctx->K;
    k->rho_inf = ctx->rho_inf;
    k->ds = ds;
    k->optics_hash = optics_hash(ctx);
    return pbr::host::field_fingerprint(ctx, &k->field_sum);
}

int sfail(pbr_surrogate *s, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_surr_create_err = buf;
    return code;
}

int shf(pbr_surrogate *s, int e, const char *what)
{
    return sfail(s, PBR_ERR_HIP, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

int64_t round64(int64_t n) { return (n + 63) / 64 * 64; }

// SplitMix64 (Steele, Lea & Flood 2014): the k-th output of the stream seeded with `seed`.
uint64_t splitmix64_host(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t seed, uint64_t k) { return (double)(splitmix64_host(seed, k) >> 11) * 0x1.0p-53; }

constexpr int kMaxTiles = 1024;  // tiles per side of the fallback map

// Consecutive 256-byte aligned parts of a caller's workspace; with a null base it only sums the
// sizes, so that one function both sizes a workspace and lays it out.
struct Carve {
    unsigned char *base = nullptr;
    size_t off = 0;
    template <typename T> T *take(size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += bytes < 256 ? 256 : bytes;
        return p;
    }
    size_t bytes() const { return (off + 255) & ~(size_t)255; }
};

int64_t rows_cap_of(int64_t max_rows) { return max_rows == 0 ? 65536 : round64(max_rows); }

// The surrogate's own device memory: FP32 parameters, gradient and Adam moments, bfloat16 weight
// copies, the training pass buffers for R rows, the inference buffers for trace chunks of `chunk`
// rays (features 24 B, outputs 24 B, eligibility 1 B and the tracer's list 4 B per ray) and the
// tile map.
void layout_persistent(pbr_surrogate *s, Carve &c, int64_t R, int64_t chunk)
{
    const int64_t H = pbr::kHidden, P = pbr::kParams + 64;
    s->d.params = c.take<float>(P * 4);
    s->d.grad = c.take<float>(P * 4);
    s->d.m = c.take<float>(P * 4);
    s->d.v = c.take<float>(P * 4);
    unsigned short **w[6] = {&s->d.w2, &s->d.w2t, &s->d.w3, &s->d.w3t, &s->d.w4, &s->d.w4t};
    for (auto q : w) *q = c.take<unsigned short>(H * H * 2);
    s->d.w5 = c.take<unsigned short>(pbr::kOutPad * H * 2);
    s->tb.rows_cap = R;
    for (int l = 0; l < 3; ++l) {
        s->tb.aT[l] = c.take<unsigned short>(H * R * 2);
        s->tb.dzT[l] = c.take<unsigned short>(H * R * 2);
    }
    s->tb.zbuf = c.take<float>((size_t)4 * R * H * 4);
    s->tb.rowpart = c.take<float>((size_t)(R / pbr::kTrainBlockRows) * pbr::kTrainPartStride * 4);
    s->tb.rowsum = c.take<float>((size_t)((R / pbr::kTrainBlockRows + 15) / 16) * pbr::kTrainPartStride * 4);
    s->tb.dwpart = c.take<float>((size_t)3 * pbr::kMaxDwSplits * H * H * 4);
    s->x = c.take<float>(R * 6 * 4);
    s->y = c.take<float>(R * 6 * 4);
    s->t = c.take<float>(R * 6 * 4);
    s->loss = c.take<float>(256);
    s->count = c.take<unsigned long long>(256);
    s->step = c.take<int>(256);
    s->tile_ok_dev = c.take<unsigned char>((size_t)kMaxTiles * kMaxTiles);
    s->ix = c.take<float>((size_t)chunk * 24);
    s->iy = c.take<float>((size_t)chunk * 24);
    s->ielig = c.take<unsigned char>((size_t)chunk);
    s->tlist = c.take<int>((size_t)chunk * 4);
    s->chunk_cap = chunk;
}

// Scratch of one pbr_surrogate_train call, carved from the caller's training workspace.
struct TrainScratch {
    pbr::SurrogateSample *trs, *vas;
    double *part;
    int *flags;      // per training ray, then per validation ray (entry tiles)
    int *perm[2];    // shuffled sample order of alternate epochs
    float *losses;
    unsigned *tile_err, *tile_cnt;
    float *err;
};

int64_t train_steps_bound(int64_t n_train, int32_t batch, int32_t epochs)
{
    return n_train / batch * (int64_t)epochs;
}

void layout_train(TrainScratch *t, Carve &c, int64_t n_train, int64_t n_val, int32_t batch, int32_t epochs,
                  int32_t tiles)
{
    const int64_t nt = (int64_t)tiles * tiles;
    t->trs = c.take<pbr::SurrogateSample>((size_t)n_train * sizeof(pbr::SurrogateSample));
    t->vas = c.take<pbr::SurrogateSample>((size_t)n_val * sizeof(pbr::SurrogateSample));
    t->part = c.take<double>((size_t)1024 * pbr::kMoments * sizeof(double));
    t->flags = c.take<int>((size_t)std::max(n_train, n_val) * sizeof(int));
    for (int b = 0; b < 2; ++b) t->perm[b] = c.take<int>((size_t)(n_train / batch * batch) * sizeof(int));
    t->losses = c.take<float>((size_t)train_steps_bound(n_train, batch, epochs) * sizeof(float));
    t->tile_err = c.take<unsigned>((size_t)(nt + 1) * 4);
    t->tile_cnt = c.take<unsigned>((size_t)(nt + 1) * 4);
    t->err = c.take<float>((size_t)n_val * 4);
}

// Default parameters: uniform in +-1/sqrt(fan_in) for the weights and biases of every layer.
void init_params(uint64_t seed, std::vector<float> &p)
{
    p.assign(pbr::kParams, 0.0f);
    const int sizes[6] = {pbr::kIn, pbr::kHidden, pbr::kHidden, pbr::kHidden, pbr::kHidden, pbr::kOut};
    int64_t o = 0;
    for (int l = 0; l < 5; ++l) {
        const double bound = 1.0 / std::sqrt((double)sizes[l]);
        const int64_t n = (int64_t)sizes[l + 1] * sizes[l] + sizes[l + 1];
        for (int64_t k = 0; k < n; ++k, ++o) p[o] = (float)((2.0 * uniform01(seed, (uint64_t)o) - 1.0) * bound);
    }
}

int check_batch(pbr_surrogate *s, const float *x, const float *t, int64_t rows)
{
    if (!x || !t) return sfail(s, PBR_ERR_ARG, "null input or target array");
    if (rows <= 0 || rows % 64 != 0 || rows > s->rows_cap)
        return sfail(s, PBR_ERR_ARG, "rows must be a positive multiple of 64 not above %lld", (long long)s->rows_cap);
    return PBR_OK;
}

// Emits and integrates n_src x rps rays without depositing them and writes one sample per ray.
int trace_samples(pbr_surrogate *s, pbr_ctx *ctx, pbr::TraceParams P, const pbr::SurrogateSpec &spec, int prec,
                  const float *src, int64_t n_src, int32_t rps, uint64_t seed, pbr::SurrogateSample *out)
{
    P.src = (const float4 *)src;
    P.n_src = n_src;
    P.rays_per_src = rps;
    P.n_rays = n_src * (int64_t)rps;
    P.seed = seed;
    P.record = 0;
    for (int64_t first = 0; first < P.n_rays; first += ctx->ray_chunk) {
        const int64_t n = std::min(ctx->ray_chunk, P.n_rays - first);
        int e = pbr::launch_trace_chunk(P, ctx->ray_ws, first, n, prec, ctx->stream, nullptr, nullptr, nullptr, false);
        if (e) return shf(s, e, "sample trace");
        if ((e = pbr::launch_surr_samples(P, spec, ctx->ray_ws, first, n, out + first, ctx->stream)))
            return shf(s, e, "sample extraction");
    }
    return PBR_OK;
}

// Per-chunk hook of a trace: the rays of eligible tiles through the network, in groups of rows_cap;
// the rest of the rays that entered the box are listed for the integration kernel.
int hook_run(void *self, const pbr::TraceParams &P, pbr::RayState *st, int64_t, int64_t n, hipStream_t stream,
             pbr::TraceList *list)
{
    pbr_surrogate *s = (pbr_surrogate *)self;
    if (n > s->chunk_cap) return (int)hipErrorInvalidValue;  // sized when the trace was validated
    int e;
    if ((e = pbr::launch_clear_u64(s->count + 1, 1, stream))) return e;
    if ((e = pbr::launch_surr_features(P, s->spec, st, n, s->ix, s->ielig, s->tlist, s->count + 1, stream)) ||
        (e = pbr::mlp_infer(s->d, s->ix, n, s->iy, stream)) ||
        (e = pbr::launch_surr_apply(P, s->spec, s->iy, s->ielig, n, st, stream)))
        return e;
    list->idx = s->tlist;
    list->count = s->count + 1;
    return 0;
}

}  // namespace

namespace pbr {
namespace host {

int surrogate_hook(pbr_ctx *ctx, double ds, int64_t chunk, ChunkHook *out)
{
    pbr_surrogate *s = ctx->surr;
    if (!s) return fail(ctx, PBR_ERR_STATE, "PBR_SURROGATE set but no surrogate attached (pbr_set_surrogate)");
    if (!s->trained || s->ctx_uid != ctx->uid || s->scene_version != ctx->scene_version)
        return fail(ctx, PBR_ERR_STATE, "the attached surrogate no longer matches this context's field, optics or sensor");
    if (ds != s->ds)
        return fail(ctx, PBR_ERR_STATE, "the surrogate was trained for steps of %.6g m, the trace asks for %.6g m", s->ds, ds);
    if (chunk > s->chunk_cap)
        return fail(ctx, PBR_ERR_WORKSPACE,
                    "the surrogate was created for trace chunks of at most %lld rays, the trace uses %lld",
                    (long long)s->chunk_cap, (long long)chunk);
    out->run = hook_run;
    out->self = s;
    return PBR_OK;
}

}  // namespace host
}  // namespace pbr

#define SURR_GUARD_BEGIN try {
#define SURR_GUARD_END                                                       \
    }                                                                        \
    catch (...) { return sfail(s, PBR_ERR_HIP, "internal error (exception)"); }

extern "C" {

size_t pbr_surrogate_workspace_bytes(int64_t max_rows, int64_t ray_chunk)
{
    if (max_rows < 0 || max_rows > ((int64_t)1 << 24) || ray_chunk < 0 || ray_chunk > ((int64_t)1 << 31)) return 0;
    pbr_surrogate probe;
    Carve c;
    layout_persistent(&probe, c, rows_cap_of(max_rows), ray_chunk);
    return c.bytes();
}

int pbr_surrogate_create(pbr_surrogate **out, int device, void *hip_stream, uint64_t init_seed, int64_t max_rows,
                         int64_t ray_chunk, void *ws_dev, size_t ws_bytes)
{
    pbr_surrogate *s = nullptr;
    try {
        if (!out) return sfail(nullptr, PBR_ERR_ARG, "out is null");
        *out = nullptr;
        if (max_rows < 0 || max_rows > ((int64_t)1 << 24))
            return sfail(nullptr, PBR_ERR_ARG, "max_rows must lie in [0, 2^24]");
        if (ray_chunk < 0 || ray_chunk > ((int64_t)1 << 31))
            return sfail(nullptr, PBR_ERR_ARG, "ray_chunk must lie in [0, 2^31]");
        if (!ws_dev || ((uintptr_t)ws_dev & 255u))
            return sfail(nullptr, PBR_ERR_ARG, "workspace must be non-null and 256-byte aligned");
        const size_t need = pbr_surrogate_workspace_bytes(max_rows, ray_chunk);
        if (ws_bytes < need)
            return sfail(nullptr, PBR_ERR_WORKSPACE, "workspace of %zu bytes < %zu", ws_bytes, need);
        int ndev = 0, e = (int)hipGetDeviceCount(&ndev);
        if (e) return sfail(nullptr, PBR_ERR_HIP, "hipGetDeviceCount: %s", hipGetErrorString((hipError_t)e));
        if (device == -1 && (e = (int)hipGetDevice(&device)))
            return sfail(nullptr, PBR_ERR_HIP, "hipGetDevice: %s", hipGetErrorString((hipError_t)e));
        if (device < 0 || device >= ndev)
            return sfail(nullptr, PBR_ERR_ARG, "device %d out of range (%d devices)", device, ndev);
        DeviceGuard g(device);
        if (!g.ok) return sfail(nullptr, PBR_ERR_HIP, "hipSetDevice(%d) failed", device);
        s = new (std::nothrow) pbr_surrogate();
        if (!s) return sfail(nullptr, PBR_ERR_HIP, "out of host memory");
        s->device = device;
        s->rows_cap = rows_cap_of(max_rows);
        s->stream = (hipStream_t)hip_stream;  // NULL: the null stream
        Carve c;
        c.base = (unsigned char *)ws_dev;
        layout_persistent(s, c, s->rows_cap, ray_chunk);
        if ((e = (int)hipStreamCreateWithFlags(&s->train_stream, hipStreamNonBlocking)) ||
            (e = (int)hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking))) {
            const int r = sfail(nullptr, PBR_ERR_HIP, "training streams: %s", hipGetErrorString((hipError_t)e));
            if (s->train_stream) (void)hipStreamDestroy(s->train_stream);
            delete s;
            return r;
        }
        *out = s;
        std::vector<float> init;
        init_params(init_seed, init);
        const int r = pbr_surrogate_set_params(s, init.data(), pbr::kParams);
        if (r) {
            g_surr_create_err = s->err;
            pbr_surrogate_destroy(s);
            *out = nullptr;
            return r;
        }
        return PBR_OK;
    } catch (...) {
        if (s) pbr_surrogate_destroy(s);
        if (out) *out = nullptr;
        return sfail(nullptr, PBR_ERR_HIP, "internal error (exception)");
    }
}

void pbr_surrogate_destroy(pbr_surrogate *s)
{
    if (!s) return;
    try {
        DeviceGuard g(s->device);
        (void)hipStreamSynchronize(s->stream);
        for (hipStream_t q : {s->train_stream, s->copy_stream})
            if (q) {
                (void)hipStreamSynchronize(q);
                (void)hipStreamDestroy(q);
            }
    } catch (...) {
    }
    delete s;
}

const char *pbr_surrogate_last_error(const pbr_surrogate *s) { return s ? s->err.c_str() : g_surr_create_err.c_str(); }

int pbr_surrogate_set_params(pbr_surrogate *s, const float *params_host, int64_t n)
{
    if (!s) return PBR_ERR_ARG;
    SURR_GUARD_BEGIN
    if (!params_host) return sfail(s, PBR_ERR_ARG, "params is null");
    if (n != pbr::kParams) return sfail(s, PBR_ERR_ARG, "expected %d parameters, got %lld", pbr::kParams, (long long)n);
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(params_host[k])) return sfail(s, PBR_ERR_ARG, "parameter %lld is not finite", (long long)k);
    DeviceGuard g(s->device);
    if (!g.ok) return sfail(s, PBR_ERR_HIP, "hipSetDevice failed");
    int e;
    if ((e = (int)hipMemcpyAsync(s->d.params, params_host, (size_t)n * 4, hipMemcpyHostToDevice, s->stream)))
        return shf(s, e, "copy parameters");
    const int64_t words = ((int64_t)pbr::kParams + 64) / 2;
    if ((e = pbr::launch_clear_u64((unsigned long long *)s->d.m, words, s->stream)) ||
        (e = pbr::launch_clear_u64((unsigned long long *)s->d.v, words, s->stream)) ||
        (e = pbr::launch_clear_u64((unsigned long long *)s->d.grad, words, s->stream)))
        return shf(s, e, "clear Adam state");
    if ((e = pbr::mlp_refresh_shadow(s->d, s->stream))) return shf(s, e, "bf16 weights");
    if ((e = (int)hipStreamSynchronize(s->stream))) return shf(s, e, "set parameters");
    s->trained = false;  // the fallback map described the previous weights
    return PBR_OK;
    SURR_GUARD_END
}

int pbr_surrogate_get_params(pbr_surrogate *s, float *params_host, int64_t n)
{
    if (!s) return PBR_ERR_ARG;
    SURR_GUARD_BEGIN
    if (!params_host) return sfail(s, PBR_ERR_ARG, "params is null");
    if (n != pbr::kParams) return sfail(s, PBR_ERR_ARG, "expected %d parameters, got %lld", pbr::kParams, (long long)n);
    DeviceGuard g(s->device);
    if (!g.ok) return sfail(s, PBR_ERR_HIP, "hipSetDevice failed");
    int e;
    if ((e = (int)hipMemcpyAsync(params_host, s->d.params, (size_t)n * 4, hipMemcpyDeviceToHost, s->stream)))
        return shf(s, e, "copy parameters");
    if ((e = (int)hipStreamSynchronize(s->stream))) return shf(s, e, "get parameters");
    return PBR_OK;
    SURR_GUARD_END
}

int pbr_surrogate_forward(pbr_surrogate *s, const float *x_dev, int64_t rows, float *y_dev)
{
    if (!s) return PBR_ERR_ARG;
    SURR_GUARD_BEGIN
    if (rows < 0) return sfail(s, PBR_ERR_ARG, "rows < 0");
    if (rows > 0 && (!x_dev || !y_dev)) return sfail(s, PBR_ERR_ARG, "null input or output array");
    DeviceGuard g(s->device);
    if (!g.ok) return sfail(s, PBR_ERR_HIP, "hipSetDevice failed");
    const int e = pbr::mlp_infer(s->d, x_dev, rows, y_dev, s->stream);
    if (e) return shf(s, e, "forward");
    return PBR_OK;
    SURR_GUARD_END
}

int pbr_surrogate_gradients(pbr_surrogate *s, const float *x_dev, const float *t_dev, int64_t rows,
                            float *grad_host, double *loss_host)
{
    if (!s) return PBR_ERR_ARG;
    SURR_GUARD_BEGIN
    int r = check_batch(s, x_dev, t_dev, rows);
    if (r) return r;
    DeviceGuard g(s->device);
    if (!g.ok) return sfail(s, PBR_ERR_HIP, "hipSetDevice failed");
    int e;
    if ((e = pbr::mlp_train_step(s->d, s->tb, x_dev, t_dev, rows, 0, 0.0f, 0, nullptr, 0, 0.0f, 0.0f, s->loss,
                                 s->stream)))
        return shf(s, e, "forward / backward");
    float l = 0.0f;
    if ((e = (int)hipMemcpyAsync(&l, s->loss, 4, hipMemcpyDeviceToHost, s->stream))) return shf(s, e, "copy loss");
    if (grad_host &&
        (e = (int)hipMemcpyAsync(grad_host, s->d.grad, (size_t)pbr::kParams * 4, hipMemcpyDeviceToHost, s->stream)))
        return shf(s, e, "copy gradients");
    if ((e = (int)hipStreamSynchronize(s->stream))) return shf(s, e, "gradients");
    if (loss_host) *loss_host = (double)l;
    return PBR_OK;
    SURR_GUARD_END
}

int pbr_surrogate_adam_step(pbr_surrogate *s, const float *x_dev, const float *t_dev, int64_t rows, float lr,
                            int32_t step, double *loss_host)
{
    if (!s) return PBR_ERR_ARG;
    SURR_GUARD_BEGIN
    int r = check_batch(s, x_dev, t_dev, rows);
    if (r) return r;
    if (!(lr > 0.0f) || !std::isfinite(lr)) return sfail(s, PBR_ERR_ARG, "lr must be finite and > 0");
    if (step < 1) return sfail(s, PBR_ERR_ARG, "step must be >= 1");
    DeviceGuard g(s->device);
    if (!g.ok) return sfail(s, PBR_ERR_HIP, "hipSetDevice failed");
    int e;
    if ((e = pbr::mlp_train_step(s->d, s->tb, x_dev, t_dev, rows, 1, lr, step, nullptr, 0, 0.0f, 0.0f, s->loss,
                                 s->stream)))
        return shf(s, e, "Adam step");
    s->trained = false;  // the fallback map no longer describes these weights
    if (loss_host) {
        float l = 0.0f;
        if ((e = (int)hipMemcpyAsync(&l, s->loss, 4, hipMemcpyDeviceToHost, s->stream))) return shf(s, e, "copy loss");
        if ((e = (int)hipStreamSynchronize(s->stream))) return shf(s, e, "Adam step");
        *loss_host = (double)l;
    }
    return PBR_OK;
    SURR_GUARD_END
}

size_t pbr_surrogate_train_workspace_bytes(int64_t n_train_rays, int64_t n_val_rays, int32_t batch, int32_t epochs,
                                           int32_t tiles)
{
    if (n_train_rays < 1 || n_val_rays < 1 || n_train_rays > ((int64_t)1 << 31) - 1 ||
        n_val_rays > ((int64_t)1 << 31) - 1 || batch < 64 || batch % 64 || epochs < 1 || tiles < 1 ||
        tiles > kMaxTiles || train_steps_bound(n_train_rays, batch, epochs) > (1ll << 30))
        return 0;
    TrainScratch t{};
    Carve c;
    layout_train(&t, c, n_train_rays, n_val_rays, batch, epochs, tiles);
    return c.bytes();
}

int pbr_surrogate_train(pbr_surrogate *s, pbr_ctx *ctx, const float *train_src_dev, int64_t n_train_src,
                        int32_t train_rays_per_src, const float *val_src_dev, int64_t n_val_src,
                        int32_t val_rays_per_src, uint64_t train_seed,
                        uint64_t val_seed, double ds, const pbr_surrogate_train_config *cfg, void *ws_dev,
                        size_t ws_bytes, pbr_surrogate_report *report)
{
    if (!s) return PBR_ERR_ARG;
    SURR_GUARD_BEGIN
    using clk = std::chrono::steady_clock;
    if (!ctx || !cfg || !report) return sfail(s, PBR_ERR_ARG, "null context, config or report");
    if (ctx->device < 0) return sfail(s, PBR_ERR_STATE, "host-only context: no device work");
    if (ctx->device != s->device) return sfail(s, PBR_ERR_ARG, "context and surrogate live on different devices");
    pbr::host::Derived dv;
    if (pbr::host::derive(ctx, &dv)) return sfail(s, PBR_ERR_STATE, "context: %s", ctx->err.c_str());
    if (ctx->has_chain) return sfail(s, PBR_ERR_STATE, "surrogate training uses the singlet (an optical chain is set)");
    if (!ctx->ray_ws) return sfail(s, PBR_ERR_STATE, "context has no trace workspace");
    if (!train_src_dev || !val_src_dev || n_train_src < 1 || n_val_src < 1 || train_rays_per_src < 1 ||
        val_rays_per_src < 1)
        return sfail(s, PBR_ERR_ARG, "need training and validation sources and rays per source >= 1");
    if (((uintptr_t)train_src_dev & 15u) || ((uintptr_t)val_src_dev & 15u))
        return sfail(s, PBR_ERR_ARG, "source arrays must be 16-byte aligned");
    const int64_t n_train = n_train_src * (int64_t)train_rays_per_src, n_val = n_val_src * (int64_t)val_rays_per_src;
    if (n_train > ((int64_t)1 << 31) - 1 || n_val > ((int64_t)1 << 31) - 1)
        return sfail(s, PBR_ERR_ARG, "at most 2^31 - 1 training and validation rays");
    if (!(ds > 0.0) || !std::isfinite(ds)) return sfail(s, PBR_ERR_ARG, "ds must be finite and > 0");
    if (cfg->batch < 64 || cfg->batch % 64 || cfg->batch > s->rows_cap)
        return sfail(s, PBR_ERR_ARG, "batch must be a multiple of 64 in [64, %lld]", (long long)s->rows_cap);
    if (cfg->epochs < 1) return sfail(s, PBR_ERR_ARG, "epochs must be >= 1");
    if (!(cfg->lr_max > 0.0f) || !(cfg->lr_min >= 0.0f) || !(cfg->lr_min <= cfg->lr_max) || !std::isfinite(cfg->lr_max))
        return sfail(s, PBR_ERR_ARG, "need 0 <= lr_min <= lr_max, lr_max > 0");
    if (!(cfg->tol_px > 0.0)) return sfail(s, PBR_ERR_ARG, "tol_px must be > 0");
    if (cfg->tiles < 1 || cfg->tiles > 1024) return sfail(s, PBR_ERR_ARG, "tiles must lie in [1, 1024]");
    if (cfg->min_tile_samples < 1) return sfail(s, PBR_ERR_ARG, "min_tile_samples must be >= 1");
    if (!ws_dev || ((uintptr_t)ws_dev & 255u))
        return sfail(s, PBR_ERR_ARG, "training workspace must be non-null and 256-byte aligned");
    {
        const size_t need = pbr_surrogate_train_workspace_bytes(n_train, n_val, cfg->batch, cfg->epochs, cfg->tiles);
        if (need == 0) return sfail(s, PBR_ERR_ARG, "too many Adam steps (rays / batch x epochs above 2^30)");
        if (ws_bytes < need)
            return sfail(s, PBR_ERR_WORKSPACE, "training workspace of %zu bytes < %zu", ws_bytes, need);
    }
    DeviceGuard g(s->device);
    if (!g.ok) return sfail(s, PBR_ERR_HIP, "hipSetDevice failed");
    std::memset(report, 0, sizeof *report);
    s->trained = false;
    if (ctx->surr == s) ctx->surr = nullptr;
    hipStream_t st = ctx->stream;
    int e;
    if ((e = (int)hipStreamSynchronize(s->stream))) return shf(s, e, "surrogate stream");

    pbr::TraceParams P;
    pbr::host::fill_params(ctx, dv, ds, &P);
    P.accum = nullptr;
    pbr::SurrogateSpec spec{};
    spec.z_lo = P.lo[2]; spec.z_hi = P.hi[2];
    spec.x_lo = P.lo[0]; spec.x_hi = P.hi[0];
    spec.y_lo = P.lo[1]; spec.y_hi = P.hi[1];
    spec.Lx = P.hi[0] - P.lo[0];
    spec.Ly = P.hi[1] - P.lo[1];
    spec.theta = 1.0;
    for (int k = 0; k < 6; ++k) { spec.t_mean[k] = 0.0f; spec.t_scale[k] = 1.0f; }
    spec.tiles = cfg->tiles;
    spec.tile_ok = nullptr;
    pbr::surrogate_spec_finish(spec);
    const int prec = ctx->n_fp64_bricks > 0 ? pbr::PREC_MIXED : pbr::PREC_FP32;

    // scratch of this call, in the caller's training workspace
    TrainScratch ts_{};
    {
        Carve c;
        c.base = (unsigned char *)ws_dev;
        layout_train(&ts_, c, n_train, n_val, cfg->batch, cfg->epochs, cfg->tiles);
    }
    pbr::SurrogateSample *trs = ts_.trs, *vas = ts_.vas;

    // 1. samples from the tracer
    auto t0 = clk::now();
    int r = trace_samples(s, ctx, P, spec, prec, train_src_dev, n_train_src, train_rays_per_src, train_seed, trs);
    if (r) return r;
    r = trace_samples(s, ctx, P, spec, prec, val_src_dev, n_val_src, val_rays_per_src, val_seed, vas);
    if (r) return r;
    // standardisation from the training samples
    double *part = ts_.part;
    int nb = 0;
    if ((e = pbr::launch_surr_moments(trs, n_train, part, &nb, st))) return shf(s, e, "moments");
    std::vector<double> hp((size_t)nb * pbr::kMoments), mom(pbr::kMoments, 0.0);
    if ((e = (int)hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st)))
        return shf(s, e, "copy moments");
    std::vector<int> flags((size_t)n_train);
    int *dflags = ts_.flags;
    if ((e = pbr::launch_surr_extract(trs, n_train, 0, dflags, st)) ||
        (e = (int)hipMemcpyAsync(flags.data(), dflags, (size_t)n_train * sizeof(int), hipMemcpyDeviceToHost, st)))
        return shf(s, e, "copy sample flags");
    if ((e = (int)hipStreamSynchronize(st))) return shf(s, e, "sample trace");
    report->sample_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < pbr::kMoments; ++k) mom[k] += hp[(size_t)b * pbr::kMoments + k];
    const double N = mom[0];
    report->train_samples = (int64_t)N;
    if (N < (double)cfg->batch)
        return sfail(s, PBR_ERR_ARG, "only %.0f training rays cross the box face to face (batch %d)", N, cfg->batch);
    for (int k = 0; k < 6; ++k) {
        const double mean = mom[1 + k] / N;
        const double var = std::max(mom[7 + k] / N - mean * mean, 0.0);
        const double sd = std::sqrt(var);
        if (sd > 1e-30) {
            spec.t_mean[k] = (float)mean;
            spec.t_scale[k] = (float)sd;
        }
    }
    spec.theta = std::sqrt((mom[13] + mom[14]) / (2.0 * N));
    if (!(spec.theta > 0.0)) spec.theta = 1.0;
    pbr::surrogate_spec_finish(spec);
    std::vector<int> valid;
    valid.reserve((size_t)N);
    for (int64_t i = 0; i < n_train; ++i)
        if (flags[(size_t)i] & 1) valid.push_back((int)i);
    std::vector<int>().swap(flags);

    // 2. Adam over shuffled batches, cosine learning rate
    const int64_t spe = (int64_t)valid.size() / cfg->batch;
    const int64_t total = spe * cfg->epochs;
    if (total > (1ll << 30)) return sfail(s, PBR_ERR_ARG, "too many Adam steps");
    float *losses = ts_.losses;
    t0 = clk::now();
    // Training steps (gather, forward, backward, loss, Adam with the step counter on the device)
    // are captured into graphs of kGraphSteps steps (and of one step for the rest of an epoch) on
    // the training stream, one set per order buffer.  The host shuffles and uploads the order of
    // epoch e + 1 on the copy stream while epoch e runs; events keep the upload behind the epoch
    // that last read its buffer and the epoch behind its upload.
    constexpr int64_t kGraphSteps = 16;
    if ((e = (int)hipStreamSynchronize(st))) return shf(s, e, "sample trace");
    hipStream_t ts = s->train_stream, cs = s->copy_stream;
    if ((e = pbr::launch_clear_u64((unsigned long long *)s->step, 1, ts))) return shf(s, e, "clear step");
    struct Resources {
        hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [order buffer][many, one]
        hipEvent_t copied[2] = {nullptr, nullptr}, done[2] = {nullptr, nullptr};
        hipStream_t ts = nullptr, cs = nullptr;
        ~Resources()
        {
            // nothing may still read or write the order buffers when the call returns
            if (ts) (void)hipStreamSynchronize(ts);
            if (cs) (void)hipStreamSynchronize(cs);
            for (auto &row : exec)
                for (hipGraphExec_t x : row)
                    if (x) (void)hipGraphExecDestroy(x);
            for (int b = 0; b < 2; ++b) {
                if (copied[b]) (void)hipEventDestroy(copied[b]);
                if (done[b]) (void)hipEventDestroy(done[b]);
            }
        }
    } rs;
    rs.ts = ts;
    rs.cs = cs;
    for (int b = 0; b < 2; ++b)
        if ((e = (int)hipEventCreateWithFlags(&rs.copied[b], hipEventDisableTiming)) ||
            (e = (int)hipEventCreateWithFlags(&rs.done[b], hipEventDisableTiming)))
            return shf(s, e, "hipEventCreate");
    const int64_t gsteps = std::min(kGraphSteps, spe);
    auto capture = [&](const int *perm, int64_t nsteps, hipGraphExec_t *exec) -> int {
        hipGraph_t graph = nullptr;
        int ce = (int)hipStreamBeginCapture(ts, hipStreamCaptureModeRelaxed);
        if (ce) return shf(s, ce, "hipStreamBeginCapture");
        for (int64_t k = 0; k < nsteps && !ce; ++k)
            if (!(ce = pbr::launch_surr_gather_step(spec, trs, perm, s->step, spe, cfg->batch, s->x, s->t, ts)))
                ce = pbr::mlp_train_step(s->d, s->tb, s->x, s->t, cfg->batch, 2, 0.0f, 0, s->step, (int)total,
                                         cfg->lr_max, cfg->lr_min, losses, ts);
        const int ee = (int)hipStreamEndCapture(ts, &graph);
        if (!ce && !ee) ce = (int)hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (ce || ee) return shf(s, ce ? ce : ee, "training step capture");
        return 0;
    };
    for (int b = 0; b < 2; ++b) {
        if ((e = capture(ts_.perm[b], gsteps, &rs.exec[b][0]))) return e;
        if (spe % gsteps && (e = capture(ts_.perm[b], 1, &rs.exec[b][1]))) return e;
    }
    const size_t order_bytes = (size_t)spe * cfg->batch * sizeof(int);
    auto shuffle = [&](int ep) {  // Fisher-Yates driven by SplitMix64, continuing from the last order
        const uint64_t es = cfg->shuffle_seed + 0x632BE59BD9B4E019ull * (uint64_t)(ep + 1);
        for (size_t i = valid.size() - 1; i > 0; --i) {
            const size_t j = (size_t)(splitmix64_host(es, i) % (uint64_t)(i + 1));
            std::swap(valid[i], valid[j]);
        }
    };
    shuffle(0);
    if ((e = (int)hipMemcpyAsync(ts_.perm[0], valid.data(), order_bytes, hipMemcpyHostToDevice, cs)) ||
        (e = (int)hipEventRecord(rs.copied[0], cs)))
        return shf(s, e, "copy order");
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        const int b = ep & 1;
        if ((e = (int)hipStreamWaitEvent(ts, rs.copied[b], 0))) return shf(s, e, "hipStreamWaitEvent");
        for (int64_t j = 0; j + gsteps <= spe; j += gsteps)
            if ((e = (int)hipGraphLaunch(rs.exec[b][0], ts))) return shf(s, e, "training steps");
        for (int64_t j = 0; j < spe % gsteps; ++j)
            if ((e = (int)hipGraphLaunch(rs.exec[b][1], ts))) return shf(s, e, "training step");
        if ((e = (int)hipEventRecord(rs.done[b], ts))) return shf(s, e, "hipEventRecord");
        if (ep + 1 == cfg->epochs) break;
        // the host order is free once its last upload has been read
        if ((e = (int)hipEventSynchronize(rs.copied[b]))) return shf(s, e, "copy order");
        shuffle(ep + 1);
        if ((e = (int)hipStreamWaitEvent(cs, rs.done[b ^ 1], 0)) ||
            (e = (int)hipMemcpyAsync(ts_.perm[b ^ 1], valid.data(), order_bytes, hipMemcpyHostToDevice, cs)) ||
            (e = (int)hipEventRecord(rs.copied[b ^ 1], cs)))
            return shf(s, e, "copy order");
    }
    if ((e = (int)hipStreamSynchronize(ts))) return shf(s, e, "training");
    std::vector<float> hl((size_t)total);
    if ((e = (int)hipMemcpy(hl.data(), losses, hl.size() * sizeof(float), hipMemcpyDeviceToHost)))
        return shf(s, e, "copy losses");
    report->train_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    report->steps = (int32_t)total;
    double l0 = 0.0, l1 = 0.0;
    for (int64_t j = 0; j < spe; ++j) {
        l0 += hl[(size_t)j];
        l1 += hl[(size_t)(total - spe + j)];
    }
    report->loss_first_epoch = l0 / (double)spe;
    report->loss_last_epoch = l1 / (double)spe;

    // 3. validation in sensor pixels, per entry tile
    t0 = clk::now();
    const int64_t nt = (int64_t)cfg->tiles * cfg->tiles;
    unsigned *tile_err = ts_.tile_err, *tile_cnt = ts_.tile_cnt;
    float *err = ts_.err;
    if ((e = pbr::launch_clear_u64((unsigned long long *)tile_err, (nt + 1) / 2, st)) ||
        (e = pbr::launch_clear_u64((unsigned long long *)tile_cnt, (nt + 1) / 2, st)))
        return shf(s, e, "clear tiles");
    for (int64_t off = 0; off < n_val; off += s->rows_cap) {
        const int64_t n = std::min(s->rows_cap, n_val - off);
        if ((e = pbr::launch_surr_gather(spec, vas + off, nullptr, n, s->x, s->t, st))) return shf(s, e, "gather");
        if ((e = pbr::mlp_infer(s->d, s->x, n, s->y, st))) return shf(s, e, "validation forward");
        if ((e = pbr::launch_surr_validate(P, spec, vas + off, s->y, n, err + off, tile_err, tile_cnt, st)))
            return shf(s, e, "validate");
    }
    std::vector<unsigned> he((size_t)nt), hc((size_t)nt);
    std::vector<float> herr((size_t)n_val);
    std::vector<int> vtile((size_t)n_val);
    int *dtile = ts_.flags;  // the training flags are consumed by now
    if ((e = pbr::launch_surr_extract(vas, n_val, 1, dtile, st))) return shf(s, e, "validation tiles");
    if ((e = (int)hipMemcpyAsync(he.data(), tile_err, (size_t)nt * 4, hipMemcpyDeviceToHost, st)) ||
        (e = (int)hipMemcpyAsync(hc.data(), tile_cnt, (size_t)nt * 4, hipMemcpyDeviceToHost, st)) ||
        (e = (int)hipMemcpyAsync(herr.data(), err, (size_t)n_val * 4, hipMemcpyDeviceToHost, st)) ||
        (e = (int)hipMemcpyAsync(vtile.data(), dtile, (size_t)n_val * sizeof(int), hipMemcpyDeviceToHost, st)))
        return shf(s, e, "copy validation");
    if ((e = (int)hipStreamSynchronize(st))) return shf(s, e, "validation");
    s->tile_ok.assign((size_t)nt, 0);
    s->tile_err.assign((size_t)nt, -1.0f);
    int32_t elig = 0;
    for (int64_t k = 0; k < nt; ++k) {
        if (!hc[(size_t)k]) continue;
        float f;
        std::memcpy(&f, &he[(size_t)k], 4);
        s->tile_err[(size_t)k] = f;
        if ((int64_t)hc[(size_t)k] >= cfg->min_tile_samples && f <= (float)cfg->tol_px) {
            s->tile_ok[(size_t)k] = 1;
            ++elig;
        }
    }
    std::vector<float> ev;
    ev.reserve((size_t)n_val);
    double max_elig = 0.0;
    int64_t n_elig = 0;
    for (int64_t i = 0; i < n_val; ++i) {
        const float x = herr[(size_t)i];
        if (x == -2.0f) ++report->val_rim_mismatches;
        if (x < 0.0f) continue;
        ev.push_back(x);
        if (s->tile_ok[(size_t)vtile[(size_t)i]]) {
            ++n_elig;
            max_elig = std::max(max_elig, (double)x);
        }
    }
    report->val_samples = (int64_t)ev.size();
    report->val_eligible = n_elig;
    report->eligible_tiles = elig;
    report->val_max_eligible_px = max_elig;
    if (!ev.empty()) {
        std::sort(ev.begin(), ev.end());
        report->val_median_px = ev[ev.size() / 2];
        report->val_p99_px = ev[std::min(ev.size() - 1, (size_t)(0.99 * (double)ev.size()))];
        report->val_max_px = ev.back();
    }
    if ((e = (int)hipMemcpy(s->tile_ok_dev, s->tile_ok.data(), (size_t)nt, hipMemcpyHostToDevice)))
        return shf(s, e, "copy tile map");
    report->validate_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    spec.tile_ok = s->tile_ok_dev;
    s->spec = spec;
    s->ds = ds;
    if (int r = scene_key(ctx, ds, &s->key)) return sfail(s, r, "field fingerprint: %s", ctx->err.c_str());
    s->ctx_uid = ctx->uid;
    s->scene_version = ctx->scene_version;
    s->trained = true;
    return PBR_OK;
    SURR_GUARD_END
}

// ------------------------------------------------------------------ save / load

}  // extern "C"

namespace {

const char kBlobMagic[8] = {'P', 'B', 'R', 'S', 'U', 'R', 'R', '1'};
constexpr uint32_t kBlobVersion = 1;

struct BlobWriter {
    std::vector<unsigned char> b;
    void put(const void *p, size_t n) { b.insert(b.end(), (const unsigned char *)p, (const unsigned char *)p + n); }
    template <typename T> void val(const T &v) { put(&v, sizeof v); }
};

struct BlobReader {
    const unsigned char *p;
    size_t n, at = 0;
    bool get(void *out, size_t k)
    {
        if (k > n - at) return false;
        std::memcpy(out, p + at, k);
        at += k;
        return true;
    }
    template <typename T> bool val(T *v) { return get(v, sizeof *v); }
};

int64_t adam_step(pbr_surrogate *s, int *out)
{
    return (int64_t)hipMemcpy(out, s->step, sizeof(int), hipMemcpyDeviceToHost);
}

// The blob: magic, version, parameter count, scene key, scaling and tile geometry, Adam step, tile
// map, per-tile validation errors, parameters, Adam moments m and v, then an FNV-1a checksum of all
// the preceding bytes.
int build_blob(pbr_surrogate *s, std::vector<unsigned char> *out)
{
    const size_t N = (size_t)pbr::kParams;
    std::vector<float> params(N), m(N), v(N);
    int step = 0;
    int e;
    if ((e = (int)hipStreamSynchronize(s->stream)) ||
        (e = (int)hipMemcpy(params.data(), s->d.params, N * 4, hipMemcpyDeviceToHost)) ||
        (e = (int)hipMemcpy(m.data(), s->d.m, N * 4, hipMemcpyDeviceToHost)) ||
        (e = (int)hipMemcpy(v.data(), s->d.v, N * 4, hipMemcpyDeviceToHost)) || (e = (int)adam_step(s, &step)))
        return shf(s, e, "copy the trained state");
    BlobWriter w;
    w.put(kBlobMagic, 8);
    w.val(kBlobVersion);
    w.val((uint32_t)N);
    w.val(s->key);
    const pbr::SurrogateSpec &sp = s->spec;
    const double g[9] = {sp.z_lo, sp.z_hi, sp.x_lo, sp.x_hi, sp.y_lo, sp.y_hi, sp.theta, sp.Lx, sp.Ly};
    w.put(g, sizeof g);
    w.put(sp.t_mean, sizeof sp.t_mean);
    w.put(sp.t_scale, sizeof sp.t_scale);
    w.val((int32_t)sp.tiles);
    w.val((int32_t)step);
    w.put(s->tile_ok.data(), s->tile_ok.size());
    w.put(s->tile_err.data(), s->tile_err.size() * 4);
    w.put(params.data(), N * 4);
    w.put(m.data(), N * 4);
    w.put(v.data(), N * 4);
    w.val(fnv1a(w.b.data(), w.b.size()));
    *out = std::move(w.b);
    return PBR_OK;
}

}  // namespace

extern "C" {

size_t pbr_surrogate_blob_bytes(pbr_surrogate *s)
{
    if (!s || !s->trained) return 0;
    const size_t nt = s->tile_ok.size();
    return 8 + 4 + 4 + sizeof(s->key) + 9 * 8 + 12 * 4 + 4 + 4 + nt * 5 + 3 * (size_t)pbr::kParams * 4 + 8;
}

int pbr_surrogate_save(pbr_surrogate *s, void *buf_host, size_t cap)
{
    if (!s) return PBR_ERR_ARG;
    SURR_GUARD_BEGIN
    if (!s->trained) return sfail(s, PBR_ERR_STATE, "surrogate not trained");
    if (!buf_host) return sfail(s, PBR_ERR_ARG, "buffer is null");
    if (cap < pbr_surrogate_blob_bytes(s))
        return sfail(s, PBR_ERR_WORKSPACE, "blob needs %zu bytes", pbr_surrogate_blob_bytes(s));
    DeviceGuard g(s->device);
    if (!g.ok) return sfail(s, PBR_ERR_HIP, "hipSetDevice failed");
    std::vector<unsigned char> b;
    if (int r = build_blob(s, &b)) return r;
    if (b.size() != pbr_surrogate_blob_bytes(s)) return sfail(s, PBR_ERR_HIP, "internal error: blob size");
    std::memcpy(buf_host, b.data(), b.size());
    return PBR_OK;
    SURR_GUARD_END
}

int pbr_surrogate_load(pbr_surrogate *s, pbr_ctx *ctx, const void *buf_host, size_t size)
{
    if (!s) return PBR_ERR_ARG;
    SURR_GUARD_BEGIN
    if (!ctx || !buf_host) return sfail(s, PBR_ERR_ARG, "null context or buffer");
    if (ctx->device < 0) return sfail(s, PBR_ERR_STATE, "host-only context: no device work");
    if (ctx->device != s->device) return sfail(s, PBR_ERR_ARG, "context and surrogate live on different devices");
    if (size < 16) return sfail(s, PBR_ERR_ARG, "blob too short");
    const unsigned char *p = (const unsigned char *)buf_host;
    uint64_t sum;
    std::memcpy(&sum, p + size - 8, 8);
    if (std::memcmp(p, kBlobMagic, 8) != 0) return sfail(s, PBR_ERR_ARG, "not a surrogate blob");
    if (fnv1a(p, size - 8) != sum) return sfail(s, PBR_ERR_ARG, "blob checksum mismatch (damaged or truncated)");
    BlobReader r{p, size - 8, 8};
    uint32_t version = 0, n_params = 0;
    pbr_surrogate::SceneKey key{};
    double g[9];
    pbr::SurrogateSpec sp{};
    int32_t tiles = 0, step = 0;
    if (!r.val(&version) || version != kBlobVersion) return sfail(s, PBR_ERR_ARG, "unsupported blob version");
    if (!r.val(&n_params) || n_params != (uint32_t)pbr::kParams) return sfail(s, PBR_ERR_ARG, "blob holds another network");
    if (!r.val(&key) || !r.get(g, sizeof g) || !r.get(sp.t_mean, sizeof sp.t_mean) ||
        !r.get(sp.t_scale, sizeof sp.t_scale) || !r.val(&tiles) || !r.val(&step))
        return sfail(s, PBR_ERR_ARG, "blob truncated");
    if (tiles < 1 || tiles > kMaxTiles) return sfail(s, PBR_ERR_ARG, "blob: bad tile count");
    const size_t nt = (size_t)tiles * (size_t)tiles, N = (size_t)pbr::kParams;
    std::vector<unsigned char> tok(nt);
    std::vector<float> terr(nt), params(N), m(N), v(N);
    if (!r.get(tok.data(), nt) || !r.get(terr.data(), nt * 4) || !r.get(params.data(), N * 4) ||
        !r.get(m.data(), N * 4) || !r.get(v.data(), N * 4) || r.at != r.n)
        return sfail(s, PBR_ERR_ARG, "blob size does not match its contents");
    // the context must hold the scene the surrogate was trained on
    pbr_surrogate::SceneKey here{};
    if (int rc = scene_key(ctx, key.ds, &here)) return sfail(s, rc, "field fingerprint: %s", ctx->err.c_str());
    if (std::memcmp(&here, &key, sizeof key) != 0)
        return sfail(s, PBR_ERR_STATE, "the context's field, optics or sensor differ from the surrogate's training scene");
    DeviceGuard dg(s->device);
    if (!dg.ok) return sfail(s, PBR_ERR_HIP, "hipSetDevice failed");
    int e;
    if ((e = (int)hipStreamSynchronize(s->stream)) ||
        (e = (int)hipMemcpy(s->d.params, params.data(), N * 4, hipMemcpyHostToDevice)) ||
        (e = (int)hipMemcpy(s->d.m, m.data(), N * 4, hipMemcpyHostToDevice)) ||
        (e = (int)hipMemcpy(s->d.v, v.data(), N * 4, hipMemcpyHostToDevice)) ||
        (e = (int)hipMemcpy(s->step, &step, sizeof step, hipMemcpyHostToDevice)))
        return shf(s, e, "copy the trained state");
    if ((e = pbr::mlp_refresh_shadow(s->d, s->stream)) || (e = (int)hipStreamSynchronize(s->stream)))
        return shf(s, e, "bf16 weights");
    if ((e = (int)hipMemcpy(s->tile_ok_dev, tok.data(), nt, hipMemcpyHostToDevice))) return shf(s, e, "copy tile map");
    sp.z_lo = g[0]; sp.z_hi = g[1]; sp.x_lo = g[2]; sp.x_hi = g[3]; sp.y_lo = g[4]; sp.y_hi = g[5];
    sp.theta = g[6]; sp.Lx = g[7]; sp.Ly = g[8];
    sp.tiles = tiles;
    pbr::surrogate_spec_finish(sp);
    sp.tile_ok = s->tile_ok_dev;
    s->spec = sp;
    s->tile_ok = std::move(tok);
    s->tile_err = std::move(terr);
    s->ds = key.ds;
    s->key = key;
    s->ctx_uid = ctx->uid;
    s->scene_version = ctx->scene_version;
    s->trained = true;
    return PBR_OK;
    SURR_GUARD_END
}

int pbr_surrogate_tile_map(pbr_surrogate *s, uint8_t *eligible_host, float *max_err_host, int64_t n_tiles)
{
    if (!s) return PBR_ERR_ARG;
    if (!s->trained) return sfail(s, PBR_ERR_STATE, "surrogate not trained");
    if (n_tiles != (int64_t)s->tile_ok.size())
        return sfail(s, PBR_ERR_ARG, "expected %lld tiles", (long long)s->tile_ok.size());
    if (eligible_host) std::memcpy(eligible_host, s->tile_ok.data(), s->tile_ok.size());
    if (max_err_host) std::memcpy(max_err_host, s->tile_err.data(), s->tile_err.size() * 4);
    return PBR_OK;
}

int pbr_set_surrogate(pbr_ctx *ctx, pbr_surrogate *s)
{
    if (!ctx) return PBR_ERR_ARG;
    if (!s) {
        ctx->surr = nullptr;
        return PBR_OK;
    }
    if (!s->trained) return pbr::host::fail(ctx, PBR_ERR_STATE, "surrogate not trained");
    if (s->ctx_uid != ctx->uid) return pbr::host::fail(ctx, PBR_ERR_STATE, "surrogate trained on another context");
    if (s->scene_version != ctx->scene_version)
        return pbr::host::fail(ctx, PBR_ERR_STATE, "field, optics or sensor changed since the surrogate was trained");
    ctx->surr = s;
    return PBR_OK;
}

}  // extern "C"
