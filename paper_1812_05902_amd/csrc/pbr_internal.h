// Internal structures shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pbr.h"

// Checked builds (compiled with -DPBR_CHECKED=1) test the index of every device access of the
// trace kernels against its buffer; regular builds leave the tests out.
#ifndef PBR_CHECKED
#define PBR_CHECKED 0
#endif

namespace pbr {

// Counter block layout (uint64 slots in the context's device block).
enum : int {
    CNT_STATUS = 0,                       // PBR_NUM_STATUS slots
    CNT_ENTERED = PBR_NUM_STATUS,         // rays that entered the box
    CNT_STEPS = PBR_NUM_STATUS + 1,       // Runge-Kutta steps
    CNT_MAXPIX = PBR_NUM_STATUS + 2,      // largest accumulator value (readout)
    CNT_STEPS64 = PBR_NUM_STATUS + 3,     // Runge-Kutta steps taken in FP64 (mixed precision)
    CNT_SURR = PBR_NUM_STATUS + 4,        // rays whose box passage the surrogate network replaced
    CNT_BAD_ACCESS = PBR_NUM_STATUS + 5,  // checked builds: device accesses found outside their buffer
    CNT_SLOTS = 16,
    CNT_QUEUE = 32                        // ray queue of the refill integration kernel (not a statistic)
};

constexpr int kMaxFootprint = 8;          // deposit window half-width limit (sigma <= 2.67 px)

// Field layout: one 128-byte record per grid cell, [nz-1][ny-1][nx-1], x fastest.  Record =
// 8 float4; float4 m holds trilinear coefficient m of the four interpolated quantities
// (n - 1, dn/dx, dn/dy, dn/dz) in its x, y, z, w lanes, so that inside the cell, at fractions
// (x, y, z) in [0, 1]^3,
//   q(x, y, z) = c0 + c1 x + c2 y + c3 z + c4 x y + c5 x z + c6 y z + c7 x y z,
// which is the trilinear interpolant of the eight corner values.
constexpr int kCellFloat4 = 8;

// Bricks of kBrick^3 cells carry the precision policy: the largest |grad n| at their nodes
// (float bits, for the steepness test) and a flag that selects FP64 integration steps.
constexpr int kBrick = 8;

// Byte layout of the field workspace: cell records, then per-brick max |grad n| (uint32 float
// bits), then per-brick FP64 flags (uint8); each part 256-byte aligned.
// nodes = 0: per-cell records (128 B per cell); nodes = 1: per-node float4 (n - 1, grad n), 16 B per
// node, from which a gather forms the same coefficients (8x less memory for fine grids).
struct FieldLayout {
    size_t cells_off, gmax_off, flags_off, total;
    int nbx, nby, nbz;
    int nodes;
    int64_t n_bricks;
};
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
inline FieldLayout field_layout(int nx, int ny, int nz, bool nodes = false)
{
    FieldLayout L;
    L.nbx = (nx - 1 + kBrick - 1) / kBrick;
    L.nby = (ny - 1 + kBrick - 1) / kBrick;
    L.nbz = (nz - 1 + kBrick - 1) / kBrick;
    L.nodes = nodes ? 1 : 0;
    L.n_bricks = (int64_t)L.nbx * L.nby * L.nbz;
    L.cells_off = 0;
    L.gmax_off = nodes ? align256((size_t)nx * (size_t)ny * (size_t)nz * 16)
                       : align256((size_t)(nx - 1) * (size_t)(ny - 1) * (size_t)(nz - 1) * kCellFloat4 * 16);
    L.flags_off = align256(L.gmax_off + (size_t)L.n_bricks * 4);
    L.total = align256(L.flags_off + (size_t)L.n_bricks);
    return L;
}

// Everything one trace launch reads.  Passed by value as the kernel argument.
struct TraceParams {
    const float4 *cells;   // field records (see above)
    const unsigned char *brick_fp64;  // per-brick FP64 flags (mixed precision)
    int nbx, nby, nbz;     // brick counts
    int nx, ny, nz;        // node counts
    int max_steps;
    double origin[3], spacing[3];
    double lo[3], hi[3];
    double step_cell[3];   // h / spacing: cell units moved per unit of T in one full step
    double h;              // step of the ray parameter t (dR/dt = T): ds / n_inf
    double n_inf;
    // sources and rays
    const float4 *src;
    const int64_t *order;  // processing order of the sources (null: index order); rays keep their keys
    int64_t n_src;
    int64_t n_rays;
    int32_t rays_per_src;
    int32_t record;        // write exit records
    uint64_t seed;
    // optics (lens frame origin: front vertex on the axis)
    double z_lens, a, R, t, clear, n_glass, z_sensor;
    // sensor
    unsigned long long *accum;
    int W, H;
    double pitch;
    double sigma_px;
    int rfp;
    int node_layout;       // field stored per node (see FieldLayout) instead of per cell
    // exit records
    pbr_ray_exit *rec;
    int64_t rec_first, rec_stride, rec_max;
    // counters
    unsigned long long *counters;
    // per-source sums of the sensor hits (null: not kept)
    pbr_source_sum *src_sums;
    // Mie weighting (null: off): intensity table at theta_k = k pi / (mie_n - 1), laser direction
    const double *mie;
    double laser[3];
    int mie_n;
    int pad1;
    // general optical chain (null: the singlet above)
    const pbr_optical_chain *chain;
    // FP32 constants of a full integration step, rounded once on the host from h and step_cell so
    // that the kernels hold them in scalar registers: g = h / spacing, g / 2, h, h / 4, h / 2,
    // h * (1/6) (float products, as the partial steps form them).  kin: per axis the cells a full
    // step may cross when |T| <= 1.05 (any gas), ceil(1.05 g + 4e-3) and at least 1; tlim32: min
    // over the axes of (kin - 4e-3) / g, the largest |T| component for which a full step from a
    // cell at least kin cells from both faces ends 4e-3 cells inside the box (see the integration
    // kernel)
    float g32[3], gh32[3];
    float h32, h4_32, h2_32, h6_32, tlim32;
    int kin[3];
};

// Offset of the optical chain inside the context's 4 KiB device block (counters come first).
constexpr size_t kChainOffset = 2048;
static_assert(kChainOffset + sizeof(pbr_optical_chain) <= 4096, "optical chain fits the device block");
static_assert(kChainOffset >= 8 * (CNT_QUEUE + 1), "optical chain after the counters");

// Per-ray state between the three trace kernels (emit -> box -> finish), 64 bytes.
// In the box: cell index c, cell fractions fd (FP64), direction T = Tr + dT (Tr at entry).
// A ray that never entered keeps its world position in fd and its unit direction as Tr + dT.
struct RayState {
    double fd[3];
    float Tr[3];
    float dT[3];
    int c[3];
    int info;  // RS_* bits, step count above RS_STEP_SHIFT
};
static_assert(sizeof(RayState) == 64, "RayState layout");
enum : int { RS_ENTERED = 1, RS_LIMITED = 2, RS_SURR = 4, RS_STEP_SHIFT = 4 };

// ---------------------------------------------------------------- ray surrogate
// Geometry of the surrogate's inputs and outputs for one field: rays enter through the box face
// z = z_lo and leave through z = z_hi.  Features: entry point scaled to [-1, 1], direction
// components over theta, sin(2 pi x / Lx), sin(2 pi y / Ly).  Targets: exit position minus the
// straight-line exit from the same entry (3), exit unit direction minus the entry direction (3),
// standardised by t_mean / t_scale.  tile_ok: eligibility over tiles x tiles of the entry face.
struct SurrogateSpec {
    double z_lo, z_hi, x_lo, x_hi, y_lo, y_hi;
    double theta, Lx, Ly;
    // reciprocals used by the kernels (set by surrogate_spec_finish): 1/(x_hi-x_lo), 1/(y_hi-y_lo),
    // 1/theta, 2 pi/Lx, 2 pi/Ly
    double inv_wx, inv_wy, inv_theta, kx, ky;
    float t_mean[6], t_scale[6];
    int tiles;
    const unsigned char *tile_ok;
};

inline void surrogate_spec_finish(SurrogateSpec &sp)
{
    sp.inv_wx = 1.0 / (sp.x_hi - sp.x_lo);
    sp.inv_wy = 1.0 / (sp.y_hi - sp.y_lo);
    sp.inv_theta = 1.0 / sp.theta;
    sp.kx = 6.283185307179586476925286766559 / sp.Lx;
    sp.ky = 6.283185307179586476925286766559 / sp.Ly;
}

// One traced ray as a training / validation sample.
struct SurrogateSample {
    float t[6];      // raw targets (metres, unit-vector components)
    int tile;        // entry tile
    int flags;       // bit 2: enters through z_lo; bit 0: and leaves through z_hi (a training
                     // sample); bit 1: the tracer's ray reaches the sensor plane through the optics
    double E[2];     // entry point (x, y) on z = z_lo
    double u[3];     // entry unit direction
    double px[2];    // tracer's sensor hit (pixels), when bit 1 is set
};
static_assert(sizeof(SurrogateSample) == 88, "SurrogateSample layout");
constexpr int kMoments = 16;  // count, sum t[6], sum t^2[6], sum u_x^2, sum u_y^2, unused

// After emission and integration of rays [first, first + n) (states st): samples out[0 .. n).
int launch_surr_samples(const TraceParams &p, const SurrogateSpec &sp, const RayState *st, int64_t first,
                        int64_t n, SurrogateSample *out, hipStream_t s);
// After emission (entry states st[0 .. n)): features of ray i in row i of x (zero rows and
// elig[i] = 0 for rays the network does not take); the other rays that entered the box are
// appended to tlist behind *tcount (which must start at zero).
int launch_surr_features(const TraceParams &p, const SurrogateSpec &sp, const RayState *st, int64_t n, float *x,
                         unsigned char *elig, int *tlist, unsigned long long *tcount, hipStream_t s);
// Writes the predicted exit state (network output row i, standardised) of every ray with elig[i].
int launch_surr_apply(const TraceParams &p, const SurrogateSpec &sp, const float *y, const unsigned char *elig,
                      int64_t n, RayState *st, hipStream_t s);
// Sensor-hit error of predictions y for samples smp[0 .. n): err[k] in pixels; 1e30 for a ray
// that entered through z_lo and left through another face; -2 when exactly one of prediction and
// tracer reaches the sensor (a rim case); -1 when neither does or the ray is not a front-face ray.
// Per-tile maxima (float bits) and counts over the err >= 0 samples, a rim case (-2) entering
// its tile as 1e30 (never eligible).
int launch_surr_extract(const SurrogateSample *smp, int64_t n, int field, int *out, hipStream_t s);
int launch_surr_validate(const TraceParams &p, const SurrogateSpec &sp, const SurrogateSample *smp,
                         const float *y, int64_t n, float *err, unsigned *tile_err, unsigned *tile_cnt,
                         hipStream_t s);
// Gathers rows idx[0 .. rows) of the samples: features into x, standardised targets into t
// (idx == nullptr: rows 0 .. rows in order).
int launch_surr_gather(const SurrogateSpec &sp, const SurrogateSample *smp, const int *idx, int64_t rows,
                       float *x, float *t, hipStream_t s);
// The same for training step *step (device): rows perm[(*step mod steps_per_epoch) * rows ..].
int launch_surr_gather_step(const SurrogateSpec &sp, const SurrogateSample *smp, const int *perm, const int *step,
                            int64_t steps_per_epoch, int64_t rows, float *x, float *t, hipStream_t s);
// Per-block sums (kMoments doubles per block) over valid samples; returns the blocks used.
int launch_surr_moments(const SurrogateSample *smp, int64_t n, double *part, int *blocks, hipStream_t s);

// Rays of a chunk left for the integration kernels: st[idx[k]] for k < *count (device values).
struct TraceList {
    const int *idx;
    const unsigned long long *count;
};

// Optional step between emission and integration of a chunk (the surrogate).  May set *list:
// then only the listed rays are integrated.
struct ChunkHook {
    int (*run)(void *self, const TraceParams &p, RayState *st, int64_t first, int64_t n, hipStream_t s,
               TraceList *list);
    void *self;
};

constexpr int kTile = 32;  // deposit pre-aggregation tile of single-image traces (pixels per side, in LDS)

// One segment of a batch round (see launch_batch_round).
struct BatchSeg {
    int32_t image;
    int32_t pad;
    int64_t first_ray;
    int64_t n_rays;
    int64_t slot_base;  // first slot (256 rays) of the segment's states in the round
};

// Tunables of the batched launch.
struct BatchConfig {
    int box_block;      // threads per block of the persistent integration kernel: 64 or 256
    int unit_rays;      // rays a wave pulls from the queue at a time: 64, 128 or 256
    int tile;           // deposit tile: 16 or 32 pixels per side
    int64_t round_rays; // rays per round (bounded by the workspace)
};

// Launchers (defined in the .hip files; enqueue on `stream`, return hipError_t as int).
// Writes the cell records and (atomically) the per-brick max |grad n|; gmax must be zeroed.
int launch_field_prep(const float *rho, float4 *cells, unsigned *brick_gmax, int nx, int ny, int nz,
                      const double spacing[3], double K, hipStream_t stream, bool nodes = false);
// Precision calibration: for each listed brick, rays_per_brick sample rays integrated over
// n_steps full steps in FP32 and in FP64 from the same state; err[k] = largest difference of
// the image point (apparent source on the plane z_focus, times |M| / pitch) in pixels.
int launch_calibrate(const TraceParams &p, const int *bricks, int n_bricks, int rays_per_brick,
                     int n_steps, uint64_t seed, double z_focus, double px_per_m, float *err,
                     hipStream_t stream);
// One round of a batch: emission over n_slots * 256 ray states, persistent integration with a
// wave-level work queue (queue: two counters, zeroed by the round, one per field layout; cells /
// nodes: the round holds images of that layout), finish with per-segment parameters.
int launch_batch_round(const TraceParams *params, const BatchSeg *segs, int nseg, int64_t n_slots,
                       RayState *st, unsigned *queue, const BatchConfig &cfg, int n_cu, hipStream_t stream,
                       bool cells, bool nodes);

// Rays [first, first + n) through all four steps; st: n RayState of workspace.
// box_begin / box_end (may be null) are recorded around the integration kernel.
enum PrecMode : int { PREC_FP32 = 0, PREC_FP64 = 1, PREC_MIXED = 2 };
int launch_trace_chunk(const TraceParams &p, RayState *st, int64_t first, int64_t n, int prec,
                       hipStream_t stream, hipEvent_t box_begin, hipEvent_t box_end,
                       const ChunkHook *hook = nullptr, bool deposit = true, bool refill = false);
int launch_readout(const unsigned long long *accum, int64_t npx, int fmt, void *out,
                   double gain, unsigned long long *counters, hipStream_t stream);
int launch_clear_u64(unsigned long long *p, int64_t n, hipStream_t stream);
// Device scratch of launch_morton_order for n sources (0 when n is out of [0, 2^31 - 1]).
size_t morton_order_scratch_bytes(int64_t n);
// order = the permutation sorting the n sources by the Morton code of their position in the box
// [lo, lo + ext] (21 bits per axis, clamped onto the box), ties in index order; ws: scratch of
// morton_order_scratch_bytes(n) bytes.
int launch_morton_order(const float4 *src, int64_t n, const double lo[3], const double ext[3], int64_t *order,
                        void *ws, hipStream_t stream);

// BOS displacement check (sec. 4).  ws: 3 uint64 per node (cleared here).
int launch_dot_map(const pbr_source_sum *with_sums, const pbr_source_sum *without_sums, const float4 *src,
                   int64_t n_src, const pbr_map_grid &g, unsigned long long *ws, float *map, hipStream_t stream);
// Eq. 9 map; scale = |M| Z_D / (n0 pitch) of the dot plane.
int launch_bos_theory(const TraceParams &p, const pbr_map_grid &g, double scale, int samples, float *map,
                      hipStream_t stream);

}  // namespace pbr
