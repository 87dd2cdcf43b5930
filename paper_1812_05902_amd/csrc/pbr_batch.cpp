// Batched rendering of many images (C ABI in include/pbr.h): host-side planning of rounds,
// capture of the whole batch into one HIP graph, and the autotuner of the batched launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "pbr_ctx.h"

struct pbr_batch {
    int device = 0;
    int n_cu = 256;
    hipStream_t stream = nullptr;      // the caller's stream: graph launches and tuning runs
    hipStream_t capture = nullptr;     // own stream the graph is captured on (the null stream cannot be)
    hipStream_t enq = nullptr;         // stream enqueue_* write to
    std::string err;
    std::vector<pbr_batch_item> items;
    std::vector<pbr::TraceParams> params;      // host copies, one per image
    std::vector<uint64_t> versions;            // each context's param_version at the snapshot
    std::vector<double> est_steps;             // cost estimate per ray, per image
    // device workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t max_round_rays = 0;
    int64_t min_round_rays = 256;
    pbr::TraceParams *d_params = nullptr;
    pbr::BatchSeg *d_segs = nullptr;
    int64_t seg_capacity = 0;
    unsigned *d_queue = nullptr;
    pbr::RayState *d_state = nullptr;
    // plan for the current configuration
    pbr::BatchConfig cfg{};
    std::vector<pbr::BatchSeg> segs;
    std::vector<int> round_begin;              // segment index of each round, plus the end
    std::vector<int64_t> round_slots;
    std::vector<unsigned char> round_layouts;  // per round: bit 0 per-cell images, bit 1 node images
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_valid = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

using pbr::host::DeviceGuard;

int bfail(pbr_batch *b, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    return code;
}

thread_local std::string g_batch_create_err;

// Workspace layout of a batch: per-image parameters, segment table, two queue counters (one per
// field layout), ray states.
struct BatchLayout {
    size_t params_off, segs_off, queue_off, state_off, total;
};

int64_t seg_capacity_for(int n_items, const int64_t *rays, int64_t round_rays)
{
    // each image splits into at most ceil(rays / round) + 1 segments (the first may share a round)
    int64_t cap = 0;
    for (int i = 0; i < n_items; ++i) cap += rays[i] / round_rays + 2;
    return cap;
}

BatchLayout batch_layout(int n_items, int64_t seg_cap, int64_t round_rays)
{
    BatchLayout L;
    L.params_off = 0;
    L.segs_off = pbr::align256((size_t)n_items * sizeof(pbr::TraceParams));
    L.queue_off = pbr::align256(L.segs_off + (size_t)seg_cap * sizeof(pbr::BatchSeg));
    L.state_off = pbr::align256(L.queue_off + 8);
    L.total = pbr::align256(L.state_off + (size_t)round_rays * sizeof(pbr::RayState));
    return L;
}

// Rounds of at most round_rays ray states: images in decreasing estimated cost per ray, each
// split across rounds as needed, each segment padded to whole 256-ray slots.
void plan(pbr_batch *b)
{
    const int n = (int)b->items.size();
    std::vector<int> order((size_t)n);
    for (int i = 0; i < n; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->est_steps[(size_t)x] > b->est_steps[(size_t)y]; });
    b->segs.clear();
    b->round_begin.assign(1, 0);
    b->round_slots.clear();
    b->round_layouts.clear();
    const int64_t cap_slots = b->cfg.round_rays / 256;
    int64_t used = 0;  // slots used in the current round
    for (int i : order) {
        const pbr_batch_item &it = b->items[(size_t)i];
        int64_t remaining = it.n_src * (int64_t)it.rays_per_src, first = 0;
        while (remaining > 0) {
            if (used == cap_slots) {
                b->round_slots.push_back(used);
                b->round_begin.push_back((int)b->segs.size());
                used = 0;
            }
            if (used == 0) b->round_layouts.push_back(0);
            b->round_layouts.back() |= b->params[(size_t)i].node_layout ? 2 : 1;
            const int64_t take = std::min(remaining, (cap_slots - used) * 256);
            pbr::BatchSeg sg;
            sg.image = i;
            sg.pad = 0;
            sg.first_ray = first;
            sg.n_rays = take;
            sg.slot_base = used;
            b->segs.push_back(sg);
            used += (take + 255) / 256;
            first += take;
            remaining -= take;
        }
    }
    if (used > 0) {
        b->round_slots.push_back(used);
        b->round_begin.push_back((int)b->segs.size());
    }
}

int upload_plan(pbr_batch *b)
{
    if ((int64_t)b->segs.size() > b->seg_capacity)
        return bfail(b, PBR_ERR_WORKSPACE, "batch plan needs %zu segments, workspace holds %lld", b->segs.size(),
                     (long long)b->seg_capacity);
    int e = 0;
    if (!b->segs.empty())
        e = (int)hipMemcpyAsync(b->d_segs, b->segs.data(), b->segs.size() * sizeof(pbr::BatchSeg),
                                hipMemcpyHostToDevice, b->stream);
    if (!e) e = (int)hipStreamSynchronize(b->stream);
    if (e) return bfail(b, PBR_ERR_HIP, "upload batch plan: %s", hipGetErrorString((hipError_t)e));
    return PBR_OK;
}

int enqueue_rounds(pbr_batch *b, int r0, int r1)
{
    for (int r = r0; r < r1; ++r) {
        const int s0 = b->round_begin[(size_t)r];
        const int ns = b->round_begin[(size_t)r + 1] - s0;
        const unsigned char lay = b->round_layouts[(size_t)r];
        const int e = pbr::launch_batch_round(b->d_params, b->d_segs + s0, ns, b->round_slots[(size_t)r],
                                              b->d_state, b->d_queue, b->cfg, b->n_cu, b->enq, (lay & 1) != 0,
                                              (lay & 2) != 0);
        if (e) return bfail(b, PBR_ERR_HIP, "batch round %d: %s", r, hipGetErrorString((hipError_t)e));
    }
    return PBR_OK;
}

// Everything one run does, in stream order: clear the requested sensors and every image's
// counters (fill kernels, no memset nodes), then all rounds.
int enqueue_batch(pbr_batch *b)
{
    for (const pbr_batch_item &it : b->items) {
        int e = 0;
        if (it.flags & PBR_CLEAR_FIRST)
            e = pbr::launch_clear_u64(it.ctx->accum, (int64_t)it.ctx->sensor.width * it.ctx->sensor.height, b->enq);
        if (!e) e = pbr::launch_clear_u64(it.ctx->counters, pbr::CNT_SLOTS, b->enq);
        if (e) return bfail(b, PBR_ERR_HIP, "batch clears: %s", hipGetErrorString((hipError_t)e));
    }
    return enqueue_rounds(b, 0, (int)b->round_slots.size());
}

void drop_graph(pbr_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_valid = false;
}

int check_config(pbr_batch *b, const pbr_batch_config *c)
{
    if (c->box_block != 64 && c->box_block != 256) return bfail(b, PBR_ERR_ARG, "box_block must be 64 or 256");
    if (c->unit_rays != 64 && c->unit_rays != 128 && c->unit_rays != 256)
        return bfail(b, PBR_ERR_ARG, "unit_rays must be 64, 128 or 256");
    if (c->tile != 16 && c->tile != 32) return bfail(b, PBR_ERR_ARG, "tile must be 16 or 32");
    if (c->round_rays < b->min_round_rays || c->round_rays % 256 != 0 || c->round_rays > b->max_round_rays)
        return bfail(b, PBR_ERR_ARG, "round_rays must be a multiple of 256 in [%lld, %lld]",
                     (long long)b->min_round_rays, (long long)b->max_round_rays);
    return PBR_OK;
}

uint64_t fnv1a(const void *p, size_t n, uint64_t h)
{
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
    return h;
}

// Key of the tuning cache: device architecture and the shape (and field layout) of every image.
std::string tune_key(pbr_batch *b)
{
    hipDeviceProp_t prop;
    uint64_t h = 0xcbf29ce484222325ull;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) h = fnv1a(prop.gcnArchName, strlen(prop.gcnArchName), h);
    for (const pbr_batch_item &it : b->items) {
        const int64_t v[8] = {it.ctx->nx, it.ctx->ny, it.ctx->nz, it.ctx->sensor.width, it.ctx->sensor.height,
                              it.n_src, it.rays_per_src, it.ctx->layout.nodes ? 1 : 0};
        h = fnv1a(v, sizeof v, h);
    }
    char buf[32];
    snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    return buf;
}

}  // namespace

extern "C" {

size_t pbr_batch_workspace_bytes(const pbr_batch_item *items, int n_items, int64_t round_rays)
{
    if (!items || n_items < 1 || round_rays < 256) return 0;
    round_rays = round_rays / 256 * 256;
    std::vector<int64_t> rays((size_t)n_items);
    for (int i = 0; i < n_items; ++i) rays[(size_t)i] = items[i].n_src * (int64_t)items[i].rays_per_src;
    const int64_t min_round = std::max<int64_t>(256, round_rays / 4 / 256 * 256);  // as pbr_batch_create
    return batch_layout(n_items, seg_capacity_for(n_items, rays.data(), min_round), round_rays).total;
}

namespace {
// The launch parameters a batch replays were taken from its contexts at creation: a context whose
// field, optics, sensor, chain or exit recording changed since then would be traced through stale
// pointers and sizes.
int check_snapshot(pbr_batch *b)
{
    for (size_t i = 0; i < b->items.size(); ++i)
        if (b->items[i].ctx->param_version != b->versions[i])
            return bfail(b, PBR_ERR_STATE,
                         "item %zu: its context's field, optics, sensor, chain or exit recording changed since "
                         "pbr_batch_create; create the batch again", i);
    return PBR_OK;
}
}  // namespace

int pbr_batch_create(pbr_batch **out, const pbr_batch_item *items, int n_items, void *ws_dev, size_t ws_bytes,
                     void *hip_stream)
{
    pbr_batch *b = nullptr;
    try {
        if (!out) { g_batch_create_err = "out is null"; return PBR_ERR_ARG; }
        *out = nullptr;
        if (!items || n_items < 1) { g_batch_create_err = "need at least one item"; return PBR_ERR_ARG; }
        if (!ws_dev || ((uintptr_t)ws_dev & 255u)) { g_batch_create_err = "workspace null or not 256-byte aligned"; return PBR_ERR_ARG; }
        b = new (std::nothrow) pbr_batch();
        if (!b) { g_batch_create_err = "out of host memory"; return PBR_ERR_HIP; }
        b->stream = (hipStream_t)hip_stream;
        b->items.assign(items, items + n_items);
        b->device = items[0].ctx ? items[0].ctx->device : -1;
        std::vector<int64_t> rays((size_t)n_items);
        for (int i = 0; i < n_items; ++i) {
            const pbr_batch_item &it = items[i];
            pbr_ctx *c = it.ctx;
            int bad = 0;
            const char *why = "";
            if (!c) { bad = PBR_ERR_ARG; why = "null context"; }
            else if (c->device < 0 || c->device != b->device) { bad = PBR_ERR_ARG; why = "contexts must share one GPU"; }
            else if (it.n_src < 0 || it.rays_per_src < 1 || (it.n_src > 0 && !it.src_dev)) { bad = PBR_ERR_ARG; why = "bad source arguments"; }
            else if (((uintptr_t)it.src_dev & 15u) != 0) { bad = PBR_ERR_ARG; why = "sources must be 16-byte aligned"; }
            else if (!(it.ds > 0.0) || !std::isfinite(it.ds)) { bad = PBR_ERR_ARG; why = "ds must be finite and > 0"; }
            else if (it.flags & ~(uint32_t)(PBR_CLEAR_FIRST | PBR_RECORD_EXITS)) { bad = PBR_ERR_ARG; why = "batch items take CLEAR_FIRST and RECORD_EXITS only (FP32 integration)"; }
            if (bad) {
                char buf[160];
                snprintf(buf, sizeof buf, "item %d: %s", i, why);
                g_batch_create_err = buf;
                delete b;
                return bad;
            }
            pbr::host::Derived d;
            const int r = pbr::host::derive(c, &d);
            if (r) { g_batch_create_err = std::string("item ") + std::to_string(i) + ": " + c->err; delete b; return r; }
            if (c->has_chain) {
                g_batch_create_err = "item " + std::to_string(i) + ": batches use the singlet (an optical chain is set)";
                delete b;
                return PBR_ERR_STATE;
            }
            const double zmax = c->origin[2] + (double)(c->nz - 1) * c->spacing[2];
            if (!(c->optics.z_front_vertex > zmax) || !(d.z_sensor > c->optics.z_front_vertex + d.t)) {
                g_batch_create_err = "item " + std::to_string(i) + ": lens must lie beyond the box, sensor behind the lens";
                delete b;
                return PBR_ERR_ARG;
            }
            rays[(size_t)i] = it.n_src * (int64_t)it.rays_per_src;
            if ((double)rays[(size_t)i] + ((it.flags & PBR_CLEAR_FIRST) ? 0.0 : c->accum_rays) > 4294967295.0) {
                g_batch_create_err = "item " + std::to_string(i) + ": more than 2^32 - 1 rays per accumulation";
                delete b;
                return PBR_ERR_OVERFLOW;
            }
            pbr::TraceParams P;
            pbr::host::fill_params(c, d, it.ds, &P);
            P.src = (const float4 *)it.src_dev;
            P.n_src = it.n_src;
            P.rays_per_src = it.rays_per_src;
            P.n_rays = rays[(size_t)i];
            P.seed = it.seed;
            P.record = (it.flags & PBR_RECORD_EXITS) && c->rec_max > 0 ? 1 : 0;
            b->params.push_back(P);
            b->versions.push_back(c->param_version);
            b->est_steps.push_back((zmax - c->origin[2]) / it.ds);  // depth of the box in steps
        }
        DeviceGuard g(b->device);
        if (!g.ok) { g_batch_create_err = "hipSetDevice failed"; delete b; return PBR_ERR_HIP; }
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && ncu > 0)
            b->n_cu = ncu;
        // the largest round R whose layout fits, with the segment table sized for rounds down to R/4
        auto min_of = [](int64_t R) { return std::max<int64_t>(256, R / 4 / 256 * 256); };
        auto fits = [&](int64_t R) {
            return batch_layout(n_items, seg_capacity_for(n_items, rays.data(), min_of(R)), R).total <= ws_bytes;
        };
        int64_t lo = 256, hi = (int64_t)(ws_bytes / sizeof(pbr::RayState)) / 256 * 256;
        if (hi < 256 || !fits(256)) {
            g_batch_create_err = "batch workspace too small";
            delete b;
            return PBR_ERR_WORKSPACE;
        }
        while (lo < hi) {
            const int64_t mid = ((lo + hi) / 2 + 255) / 256 * 256;
            if (fits(mid)) lo = mid;
            else hi = mid - 256;
        }
        b->max_round_rays = lo;
        b->min_round_rays = min_of(lo);
        b->seg_capacity = seg_capacity_for(n_items, rays.data(), b->min_round_rays);
        const BatchLayout L = batch_layout(n_items, b->seg_capacity, lo);
        b->ws = (char *)ws_dev;
        b->ws_bytes = ws_bytes;
        b->d_params = (pbr::TraceParams *)(b->ws + L.params_off);
        b->d_segs = (pbr::BatchSeg *)(b->ws + L.segs_off);
        b->d_queue = (unsigned *)(b->ws + L.queue_off);
        b->d_state = (pbr::RayState *)(b->ws + L.state_off);
        int e = (int)hipMemcpyAsync(b->d_params, b->params.data(), b->params.size() * sizeof(pbr::TraceParams),
                                    hipMemcpyHostToDevice, b->stream);
        if (!e) e = (int)hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
        if (!e) e = (int)hipEventCreate(&b->ev0);
        if (!e) e = (int)hipEventCreate(&b->ev1);
        if (e) { g_batch_create_err = std::string("batch set-up: ") + hipGetErrorString((hipError_t)e); delete b; return PBR_ERR_HIP; }
        b->enq = b->stream;
        b->cfg.box_block = 64;
        b->cfg.unit_rays = 64;
        b->cfg.tile = pbr::kTile;
        b->cfg.round_rays = b->max_round_rays;
        plan(b);
        const int r = upload_plan(b);
        if (r) { g_batch_create_err = b->err; delete b; return r; }
        *out = b;
        return PBR_OK;
    } catch (...) {
        delete b;
        g_batch_create_err = "internal error (exception)";
        return PBR_ERR_HIP;
    }
}

void pbr_batch_destroy(pbr_batch *b)
{
    if (!b) return;
    try {
        DeviceGuard g(b->device);
        (void)hipStreamSynchronize(b->stream);
        drop_graph(b);
        if (b->ev0) (void)hipEventDestroy(b->ev0);
        if (b->ev1) (void)hipEventDestroy(b->ev1);
        if (b->capture) (void)hipStreamDestroy(b->capture);
    } catch (...) {
    }
    delete b;
}

const char *pbr_batch_last_error(const pbr_batch *b) { return b ? b->err.c_str() : g_batch_create_err.c_str(); }

int pbr_batch_get_config(pbr_batch *b, pbr_batch_config *out)
{
    if (!b || !out) return PBR_ERR_ARG;
    out->box_block = b->cfg.box_block;
    out->unit_rays = b->cfg.unit_rays;
    out->tile = b->cfg.tile;
    out->reserved = 0;
    out->round_rays = b->cfg.round_rays;
    out->max_round_rays = b->max_round_rays;
    out->min_round_rays = b->min_round_rays;
    out->rounds = (int32_t)b->round_slots.size();
    return PBR_OK;
}

int pbr_batch_configure(pbr_batch *b, const pbr_batch_config *c)
{
    if (!b) return PBR_ERR_ARG;
    try {
        if (!c) return bfail(b, PBR_ERR_ARG, "config is null");
        int r = check_config(b, c);
        if (r) return r;
        DeviceGuard g(b->device);
        if (!g.ok) return bfail(b, PBR_ERR_HIP, "hipSetDevice failed");
        (void)hipStreamSynchronize(b->stream);
        drop_graph(b);
        b->cfg.box_block = c->box_block;
        b->cfg.unit_rays = c->unit_rays;
        b->cfg.tile = c->tile;
        b->cfg.round_rays = c->round_rays;
        plan(b);
        return upload_plan(b);
    } catch (...) {
        return bfail(b, PBR_ERR_HIP, "internal error (exception)");
    }
}

int pbr_batch_run(pbr_batch *b, pbr_batch_stats *stats)
{
    if (!b) return PBR_ERR_ARG;
    try {
        if (int r = check_snapshot(b)) return r;
        DeviceGuard g(b->device);
        if (!g.ok) return bfail(b, PBR_ERR_HIP, "hipSetDevice failed");
        for (size_t i = 0; i < b->items.size(); ++i) {  // overflow bound of accumulating items
            const pbr_batch_item &it = b->items[i];
            const double before = (it.flags & PBR_CLEAR_FIRST) ? 0.0 : it.ctx->accum_rays;
            if (before + (double)b->params[i].n_rays > 4294967295.0)
                return bfail(b, PBR_ERR_OVERFLOW, "item %zu: more than 2^32 - 1 rays per accumulation", i);
        }
        int e;
        if (!b->graph_valid) {
            e = (int)hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed);
            if (e) return bfail(b, PBR_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString((hipError_t)e));
            b->enq = b->capture;
            const int r = enqueue_batch(b);
            b->enq = b->stream;
            hipGraph_t graph = nullptr;
            e = (int)hipStreamEndCapture(b->capture, &graph);
            if (r) { if (graph) (void)hipGraphDestroy(graph); return r; }
            if (e) return bfail(b, PBR_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString((hipError_t)e));
            b->graph = graph;
            e = (int)hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
            if (e) { drop_graph(b); return bfail(b, PBR_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString((hipError_t)e)); }
            b->graph_valid = true;
        }
        if (stats && (e = (int)hipEventRecord(b->ev0, b->stream))) return bfail(b, PBR_ERR_HIP, "hipEventRecord");
        e = (int)hipGraphLaunch(b->exec, b->stream);
        if (e) return bfail(b, PBR_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString((hipError_t)e));
        if (stats && (e = (int)hipEventRecord(b->ev1, b->stream))) return bfail(b, PBR_ERR_HIP, "hipEventRecord");
        for (size_t i = 0; i < b->items.size(); ++i) {
            pbr_ctx *c = b->items[i].ctx;
            c->accum_rays = ((b->items[i].flags & PBR_CLEAR_FIRST) ? 0.0 : c->accum_rays) + (double)b->params[i].n_rays;
        }
#if PBR_CHECKED
        if ((e = (int)hipStreamSynchronize(b->stream)))
            return bfail(b, PBR_ERR_HIP, "batch (stream synchronise): %s", hipGetErrorString((hipError_t)e));
        for (size_t i = 0; i < b->items.size(); ++i) {
            unsigned long long bad = 0;
            e = (int)hipMemcpy(&bad, b->items[i].ctx->counters + pbr::CNT_BAD_ACCESS, sizeof bad, hipMemcpyDeviceToHost);
            if (e) return bfail(b, PBR_ERR_HIP, "read counters: %s", hipGetErrorString((hipError_t)e));
            if (bad)
                return bfail(b, PBR_ERR_BOUNDS, "checked build: image %zu made %llu device accesses outside their "
                             "buffers (clamped or skipped)", i, bad);
        }
#endif
        if (stats) {
            std::memset(stats, 0, sizeof *stats);
            e = (int)hipStreamSynchronize(b->stream);
            if (e) return bfail(b, PBR_ERR_HIP, "batch (stream synchronise): %s", hipGetErrorString((hipError_t)e));
            float ms = 0.0f;
            if ((e = (int)hipEventElapsedTime(&ms, b->ev0, b->ev1))) return bfail(b, PBR_ERR_HIP, "hipEventElapsedTime");
            stats->run_ms = (double)ms;
            stats->rounds = (int32_t)b->round_slots.size();
            stats->images = (int32_t)b->items.size();
            for (size_t i = 0; i < b->items.size(); ++i) {
                unsigned long long h[pbr::CNT_SLOTS];
                e = (int)hipMemcpy(h, b->items[i].ctx->counters, sizeof h, hipMemcpyDeviceToHost);
                if (e) return bfail(b, PBR_ERR_HIP, "read counters: %s", hipGetErrorString((hipError_t)e));
                stats->rays += (uint64_t)b->params[i].n_rays;
                for (int k = 0; k < PBR_NUM_STATUS; ++k) stats->status[k] += h[pbr::CNT_STATUS + k];
                stats->rkn_steps += h[pbr::CNT_STEPS];
                if (b->params[i].node_layout) stats->rkn_steps_nodes += h[pbr::CNT_STEPS];
            }
        }
        return PBR_OK;
    } catch (...) {
        return bfail(b, PBR_ERR_HIP, "internal error (exception)");
    }
}

int pbr_batch_autotune(pbr_batch *b, const char *cache_path, int32_t probe_rounds, pbr_batch_config *chosen,
                       double *rays_per_ms)
{
    if (!b) return PBR_ERR_ARG;
    try {
        if (int r = check_snapshot(b)) return r;
        const std::string key = tune_key(b);
        if (cache_path) {  // cached choice for this device and batch shape
            std::ifstream in(cache_path);
            std::string line;
            while (std::getline(in, line)) {
                std::istringstream ls(line);
                std::string k;
                pbr_batch_config c{};
                double rate = 0.0;
                if (ls >> k >> c.box_block >> c.unit_rays >> c.tile >> c.round_rays >> rate && k == key &&
                    check_config(b, &c) == PBR_OK) {
                    const int r = pbr_batch_configure(b, &c);
                    if (r) return r;
                    if (chosen) pbr_batch_get_config(b, chosen);
                    if (rays_per_ms) *rays_per_ms = rate;
                    return PBR_OK;
                }
            }
        }
        if (probe_rounds < 1) probe_rounds = 1;
        DeviceGuard g(b->device);
        if (!g.ok) return bfail(b, PBR_ERR_HIP, "hipSetDevice failed");
        std::vector<int64_t> rounds_rays{b->max_round_rays};
        const int64_t half = b->max_round_rays / 2 / 256 * 256;
        if (half >= b->min_round_rays && half >= 65536) rounds_rays.push_back(half);
        // every candidate: one warm-up pass over the probe rounds, then the median rate of three
        // timed passes; the three best are timed again (median of five) and the best of those kept,
        // so that one noisy timing does not decide
        struct Cand {
            pbr_batch_config c;
            double rate;
        };
        std::vector<Cand> cands;
        auto time_config = [&](const pbr_batch_config &c, int repeats, double *rate) -> int {
            int r = pbr_batch_configure(b, &c);
            if (r) return r;
            const int nr = std::min<int>(probe_rounds, (int)b->round_slots.size());
            int64_t rays = 0;
            for (int q = 0; q < nr; ++q)
                for (int s2 = b->round_begin[(size_t)q]; s2 < b->round_begin[(size_t)q + 1]; ++s2)
                    rays += b->segs[(size_t)s2].n_rays;
            if ((r = enqueue_rounds(b, 0, nr))) return r;  // warm-up (direct launches)
            std::vector<double> rates;
            for (int t = 0; t < repeats; ++t) {
                int e = (int)hipEventRecord(b->ev0, b->stream);
                if (!e && (r = enqueue_rounds(b, 0, nr))) return r;
                if (!e) e = (int)hipEventRecord(b->ev1, b->stream);
                if (!e) e = (int)hipEventSynchronize(b->ev1);
                float ms = 0.0f;
                if (!e) e = (int)hipEventElapsedTime(&ms, b->ev0, b->ev1);
                if (e) return bfail(b, PBR_ERR_HIP, "autotune timing: %s", hipGetErrorString((hipError_t)e));
                rates.push_back(ms > 0.0f ? (double)rays / (double)ms : 0.0);
            }
            std::sort(rates.begin(), rates.end());
            *rate = rates[rates.size() / 2];
            return PBR_OK;
        };
        for (int64_t rr : rounds_rays)
            for (int bb : {64, 256})
                for (int ur : {64, 256})
                    for (int tl : {16, 32}) {
                        pbr_batch_config c{};
                        c.box_block = bb;
                        c.unit_rays = ur;
                        c.tile = tl;
                        c.round_rays = rr;
                        double rate = 0.0;
                        if (int r = time_config(c, 3, &rate)) return r;
                        cands.push_back({c, rate});
                    }
        std::stable_sort(cands.begin(), cands.end(), [](const Cand &x, const Cand &y) { return x.rate > y.rate; });
        pbr_batch_config best = cands[0].c;
        double best_rate = -1.0;
        for (size_t k = 0; k < std::min<size_t>(3, cands.size()); ++k) {
            double rate = 0.0;
            if (int r = time_config(cands[k].c, 5, &rate)) return r;
            if (rate > best_rate) { best_rate = rate; best = cands[k].c; }
        }
        int r = pbr_batch_configure(b, &best);
        if (r) return r;
        if (cache_path) {
            std::ofstream outf(cache_path, std::ios::app);
            outf << key << ' ' << best.box_block << ' ' << best.unit_rays << ' ' << best.tile << ' '
                 << best.round_rays << ' ' << best_rate << '\n';
        }
        if (chosen) pbr_batch_get_config(b, chosen);
        if (rays_per_ms) *rays_per_ms = best_rate;
        return PBR_OK;
    } catch (...) {
        return bfail(b, PBR_ERR_HIP, "internal error (exception)");
    }
}

}  // extern "C"
