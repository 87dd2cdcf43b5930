/*
 * pbr.h -- C ABI of the MI355X (gfx950) ray-tracing library for synthetic PIV / BOS images.
 *
 * The library renders the image-generation method of Rajendran, Bane & Vlachos (arXiv
 * 1812.05902, section 3): rays are emitted from particles or dots towards the camera lens
 * (sec. 3.1), integrated through a 3-D refractive-index grid with the Runge-Kutta scheme of
 * eqs. 3-6 (sec. 3.2), refracted through a thick lens by Snell's law, eq. 7 (sec. 3.3), and
 * deposited into sensor pixels as error-function-integrated Gaussian spots whose diameter
 * follows eq. 8 (sec. 3.4).
 *
 * Conventions shared by every call:
 *   - Units are SI (metres, kg/m^3).  The optical axis is +z and light travels towards +z:
 *     sources, then the density box, then the lens (front vertex at pbr_optics.z_front_vertex),
 *     then the sensor.  x and y are centred on the axis.  Pixel (i, j) covers
 *     [i, i+1) x [j, j+1) in sensor pixel coordinates x_px = x / pitch + width / 2 (same for y);
 *     the image is not flipped (a real image is inverted).
 *   - "_dev" pointers are device memory of the context's GPU, owned by the caller.  The library
 *     never allocates large buffers: the caller provides the field workspace, the trace
 *     workspace, the sensor accumulator, the ray-exit record buffer, batch workspaces and the
 *     surrogate's persistent and training workspaces.  pbr_create allocates one 4 KiB device
 *     block for counters and the optical chain, freed by pbr_destroy; the calibration probes at
 *     the end allocate and free their own buffers.
 *   - All device work is enqueued on the context's HIP stream and is asynchronous unless a
 *     function says it synchronises.  The caller keeps its buffers alive until the stream has
 *     passed the work that uses them.
 *   - Every int-returning function returns PBR_OK (0) or a negative PBR_ERR_* code, and leaves a
 *     message for pbr_last_error.  Arguments are validated before any device work is enqueued,
 *     so a failed call has no effect on the device.  No C++ exception crosses the ABI.
 *   - One context per host thread and stream; contexts are independent.
 */
#ifndef PBR_H
#define PBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- return codes */
#define PBR_OK             0
#define PBR_ERR_ARG       -1  /* an argument is null, non-finite or out of range */
#define PBR_ERR_STATE     -2  /* call order: e.g. trace before field, optics or sensor are set */
#define PBR_ERR_HIP       -3  /* a HIP runtime call failed (message names it) */
#define PBR_ERR_WORKSPACE -4  /* a caller buffer is smaller than required */
#define PBR_ERR_OVERFLOW  -5  /* the 64-bit fixed-point sensor could overflow */
#define PBR_ERR_BOUNDS    -6  /* checked builds only: a trace kernel met an index outside its buffer */

/* ---------------------------------------------------------------- per-ray status */
#define PBR_RAY_DEPOSITED        0  /* reached the sensor; spot deposited */
#define PBR_RAY_OFF_SENSOR       1  /* hit point outside the pixel array */
#define PBR_RAY_BLOCKED_APERTURE 2  /* crossed the aperture plane outside the opening (sec. 3.3 (3)) */
#define PBR_RAY_BLOCKED_LENS     3  /* missed a lens surface or crossed it outside its clear radius */
#define PBR_RAY_TIR              4  /* total internal reflection inside the lens (sec. 3.3 (2)) */
#define PBR_RAY_STEP_LIMIT       5  /* exceeded the integration step limit inside the box */
#define PBR_RAY_MISSED           6  /* never travels towards the lens or the sensor */
#define PBR_NUM_STATUS           7

/* ---------------------------------------------------------------- pbr_emit_and_trace flags */
#define PBR_CLEAR_FIRST     (1u << 0)  /* zero the sensor accumulator before depositing */
#define PBR_RECORD_EXITS    (1u << 1)  /* write exit records for the rays chosen by pbr_set_exit_recording */
#define PBR_PREC_FP64_ALL   (1u << 2)  /* integrate every step in FP64 (default: FP32) */
#define PBR_PREC_SHOCK_FP64 (1u << 3)  /* FP64 steps inside the bricks flagged by pbr_calibrate_precision */
#define PBR_SURROGATE       (1u << 4)  /* rays entering through eligible tiles take the attached surrogate's exit */
#define PBR_LANE_REFILL     (1u << 5)  /* FP32 integration by persistent waves whose lanes take a new ray as
                                          soon as theirs leaves the box, instead of one thread per ray; same
                                          results bit for bit.  Off by default: lanes then hold rays of
                                          different sources, which costs more cell gathers than the idle
                                          lanes it saves (measured 4% slower on the 128^3 BOS scene, 16% on
                                          the 512^3 Tomo-PIV scene) */
#define PBR_MIE             (1u << 7)  /* weight every ray by the Mie intensity set by pbr_set_mie (sec. 3.1) */
#define PBR_SOURCE_SUMS     (1u << 6)  /* add every deposited ray's sensor hit into the per-source sums set by
                                          pbr_set_source_sums (sec. 4: a dot's displacement is the mean of
                                          its rays') */
#define PBR_SOURCE_ORDER    (1u << 8)  /* trace the sources in the order set by pbr_set_source_order; every
                                          ray keeps its key, so the results are the same bit for bit */

/* ---------------------------------------------------------------- pbr_read_image formats */
#define PBR_FMT_RAW_U64 0  /* copy of the Q32.32 accumulator (uint64 per pixel) */
#define PBR_FMT_F32     1  /* float: accumulator * 2^-32 (sum of spot fractions times weights) */
#define PBR_FMT_U16     2  /* uint16: min(65535, round_half_even(value * gain)) */

/* Camera lens: a symmetric biconvex singlet whose two radii follow from the thick-lens
 * lensmaker equation for the nominal focal length (glass index relative to vacuum); the aperture
 * stop is a disk of radius focal_length / (2 f_number) in the plane of the front vertex.  The
 * medium on both sides has the ambient index 1 + K rho_inf of pbr_set_density_field. */
typedef struct pbr_optics {
    double z_front_vertex;  /* z of the first lens surface on the axis (m) */
    double focal_length;    /* nominal focal length (m), > 0 */
    double f_number;        /* f/#, > 0; aperture radius a = focal_length / (2 f_number) */
    double thickness;       /* centre thickness (m); <= 0 selects 0.1 * focal_length */
    double n_glass;         /* lens index (> 1), e.g. 1.5 */
    double clear_radius;    /* surface clear radius (m); <= 0 selects 1.5 a */
    double z_focus;         /* object plane imaged sharply when the sensor is auto-placed */
} pbr_optics;

/* Sensor: pixel array, its plane, and the diffraction spot of eq. 8. */
typedef struct pbr_sensor {
    int32_t width, height;  /* pixels, 1 .. 16384 each */
    double pitch;           /* pixel pitch (m), > 0 */
    double z_sensor;        /* sensor plane z (m); NaN = paraxial image plane of z_focus */
    double wavelength;      /* (m), e.g. 532e-9 (effective green) */
    double sigma_px;        /* Gaussian sigma in pixels; <= 0 = d_tau / 4 from eq. 8 */
    int32_t dtau_with_pi;   /* 1: keep the factor pi printed in eq. 8; 0: d_tau = 2.44 f# (|M|+1) lambda */
    int32_t reserved;
} pbr_sensor;

/* Quantities derived by the library from field, optics and sensor (for checks and reports). */
typedef struct pbr_derived {
    double n_inf;           /* ambient refractive index 1 + K rho_inf */
    double lens_radius;     /* |R1| = |R2| (m) */
    double thickness;       /* lens centre thickness (m) */
    double aperture_radius; /* a (m) */
    double clear_radius;    /* (m) */
    double z_sensor;        /* sensor plane actually used (m) */
    double magnification;   /* paraxial lateral magnification (negative: inverted image) */
    double sigma_px;        /* spot sigma actually used (pixels) */
    int32_t footprint_r;    /* deposit window half-width: max(1, ceil(3 sigma_px)) */
    int32_t max_steps;      /* step limit for the last traced ds */
} pbr_derived;

/* Counters of one pbr_emit_and_trace call. */
typedef struct pbr_stats {
    uint64_t rays;                     /* rays emitted */
    uint64_t status[PBR_NUM_STATUS];   /* rays per PBR_RAY_* status (sums to rays) */
    uint64_t entered_volume;           /* rays that entered the density box */
    uint64_t rkn_steps;                /* Runge-Kutta steps taken (all rays) */
    uint64_t rkn_steps_fp64;           /* of which in FP64 */
    double trace_ms;                   /* device time of the whole trace (HIP events) */
    double box_ms;                     /* device time of the integration kernel launches alone */
    uint64_t box_launches;             /* integration kernel launches (one per ray chunk) */
    uint64_t surrogate_rays;           /* rays whose box passage the surrogate network replaced */
} pbr_stats;

/* Exit record of one ray (sec. 4 uses per-ray displacements on the sensor). */
typedef struct pbr_ray_exit {
    int64_t ray_id;          /* s * rays_per_src + j */
    int32_t status;          /* PBR_RAY_* */
    int32_t n_steps;         /* Runge-Kutta steps inside the box */
    int32_t entered;         /* 1 if the ray entered the density box */
    int32_t reserved;
    double vol_exit_pos[3];  /* where the ray left the box (the source if it never entered) */
    double vol_exit_dir[3];  /* unit direction there */
    double sensor_px[2];     /* hit point in pixel coordinates (valid for DEPOSITED / OFF_SENSOR) */
} pbr_ray_exit;

/* Result of pbr_calibrate_precision.  A brick is kBrick^3 = 8^3 cells. */
typedef struct pbr_precision_report {
    int64_t n_bricks;        /* bricks of the grid */
    int64_t n_steep;         /* bricks whose largest node |grad n| >= steep_frac * grid maximum */
    int64_t n_fp64;          /* steep bricks whose FP32 error exceeded tol_px: FP64 steps there */
    double grad_threshold;   /* |grad n| of the steepness test (1/m) */
    double grad_max;         /* largest node |grad n| of the grid (1/m) */
    double max_err_px;       /* largest measured FP32-vs-FP64 difference over steep bricks (pixels) */
    double tol_px;
    int32_t steps_per_sample;
    int32_t rays_per_brick;
} pbr_precision_report;

/* ---------------------------------------------------------------- context */

typedef struct pbr_ctx pbr_ctx;

/* Creates a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t; NULL =
 * the null stream).  Allocates a 4 KiB device block for counters and the optical chain.  *out is NULL on failure.
 * device = -1 creates a host-only context: every input is validated and pbr_get_derived works,
 * but no device memory is touched (pbr_set_density_field records the grid without launching) and
 * calls that need device work (trace, readout, record copies) return PBR_ERR_STATE after their
 * argument checks.  Errors: ARG (out null, device out of range), HIP. */
int pbr_create(pbr_ctx **out, int device, void *hip_stream);

/* Waits for the context's stream, frees its counter block and the context. NULL is a no-op. */
void pbr_destroy(pbr_ctx *ctx);

/* Message of the last failed call on this context (or of the last failed pbr_create when ctx is
 * NULL).  The string lives until the next call on the context. */
const char *pbr_last_error(const pbr_ctx *ctx);

/* Changes the stream later calls enqueue on. */
int pbr_set_stream(pbr_ctx *ctx, void *hip_stream);

/* 1 if this copy of the library is the checked build, 0 for the regular one.  The checked build
 * (libpbr_checked.so, a debugging aid: same entry points, same results) tests the index of every
 * device access of the trace kernels against its buffer: field gathers (per cell and per node),
 * brick flags, sources, source-order entries, the Mie table, sensor pixels and per-source sums.
 * An access that fails its test is counted, then clamped into its buffer or skipped, and
 * pbr_emit_and_trace, pbr_emit_and_trace_noalloc, pbr_calibrate_precision and pbr_batch_run return
 * PBR_ERR_BOUNDS with the count in the message after the work (they synchronise the stream to read
 * it). */
int pbr_checked_build(void);

/* ---------------------------------------------------------------- inputs */

/* Bytes of field workspace pbr_set_density_field needs for an nx x ny x nz grid: 128 bytes per
 * cell plus 5 bytes per brick of 8^3 cells, each part rounded up to 256 bytes (0 if a dimension
 * is below 2). */
size_t pbr_field_workspace_bytes(int nx, int ny, int nz);

/* Density grid (sec. 3.2 and Gladstone-Dale eq. 1).  rho_dev: float32 [nz][ny][nx] node values,
 * x fastest; node (i,j,k) sits at origin + (i,j,k) * spacing.  Enqueues the field preparation
 * kernel, which forms n - 1 = K rho and grad n at the nodes (central differences inside,
 * second-order one-sided differences on the faces) and writes, for every cell, the coefficients
 * of the trilinear interpolant of these four quantities (128 bytes per cell) into ws_dev
 * (ws_bytes >= pbr_field_workspace_bytes, 16-byte aligned).  rho_dev may be released once the
 * stream has passed this call; ws_dev must live as long as the context traces with this field.
 * Outside the box the index is 1 + K rho_inf with no gradient.  The density values are checked on
 * the device first (the call synchronises the stream for that check).
 * Errors: ARG (null, dims < 2 or > 65535, more than 2^31 - 1 cells, spacing <= 0, K < 0,
 * non-finite origin/spacing/K/rho_inf, a non-finite density value), WORKSPACE, HIP. */
int pbr_set_density_field(pbr_ctx *ctx, const float *rho_dev, int nx, int ny, int nz,
                          const double origin[3], const double spacing[3], double K,
                          double rho_inf, void *ws_dev, size_t ws_bytes);

/* Node layout for fine grids: the same field stored as one float4 (n - 1, grad n) per node (16 bytes
 * per node instead of 128 per cell, so the field of a grid whose cells are about one step long can
 * stay in the GPU's caches); the integration kernel interpolates the eight corners of the cell a
 * sample lies in directly (a dedicated kernel variant at four waves per SIMD).  Same arguments,
 * validation and results (to float32 rounding) as pbr_set_density_field; workspace
 * pbr_field_workspace_bytes_nodes: 16 bytes per node plus the brick tables, each part rounded up to
 * 256 bytes.  Lane refill (PBR_LANE_REFILL) needs the per-cell field and returns STATE with a
 * node-layout field; the precision calibration and shock FP64 steps take either layout, and so do
 * batches, image by image. */
size_t pbr_field_workspace_bytes_nodes(int nx, int ny, int nz);
int pbr_set_density_field_nodes(pbr_ctx *ctx, const float *rho_dev, int nx, int ny, int nz,
                                const double origin[3], const double spacing[3], double K,
                                double rho_inf, void *ws_dev, size_t ws_bytes);

/* Bytes of trace workspace for chunks of rays_per_chunk rays (64 bytes per ray, at least 256
 * rays).  The trace runs the rays of a call in chunks of this size through three kernels
 * (emission and box entry, ray-equation integration, lens / sensor / deposit) that hand the ray
 * state over in this workspace. */
size_t pbr_trace_workspace_bytes(int64_t rays_per_chunk);

/* Sets the trace workspace (device, 16-byte aligned, >= pbr_trace_workspace_bytes(256) bytes;
 * the chunk is ws_bytes / 64 rays).  It must live as long as traces use it.
 * Errors: ARG (null, misaligned), WORKSPACE (too small). */
int pbr_set_trace_workspace(pbr_ctx *ctx, void *ws_dev, size_t ws_bytes);

/* Lens (sec. 3.3).  Copied; host-side set-up only.  Errors: ARG (null, focal_length <= 0,
 * f_number <= 0, n_glass <= 1, thickness > n_glass * focal_length (no real lens radius),
 * clear radius < aperture radius, non-finite values). */
int pbr_set_optics(pbr_ctx *ctx, const pbr_optics *optics);

/* Sensor (sec. 3.4) and its accumulator: uint64 [height][width] Q32.32 fixed point, owned by
 * the caller, width * height * 8 bytes.  Deposits are integer atomics, so images do not depend on
 * the order in which rays arrive.  Errors: ARG. */
int pbr_set_sensor(pbr_ctx *ctx, const pbr_sensor *sensor, uint64_t *accum_dev);

/* Fills *out with the derived optics; needs field (for n_inf), optics and sensor.  Host only. */
int pbr_get_derived(pbr_ctx *ctx, pbr_derived *out);

/* Chooses the rays whose exit records later traces with PBR_RECORD_EXITS write: ray ids
 * first + k * stride for 0 <= k < max_records, record k at buf_dev[k] (caller-owned device
 * buffer of max_records pbr_ray_exit).  Records of ids beyond the traced ray count are left
 * untouched.  Errors: ARG (first < 0, stride < 1, max_records < 0, null buffer with
 * max_records > 0). */
int pbr_set_exit_recording(pbr_ctx *ctx, int64_t first, int64_t stride, int64_t max_records,
                           pbr_ray_exit *buf_dev);

/* ---------------------------------------------------------------- the hot path */

/* Emits rays_per_src rays from each of n_src sources and accumulates their spots into the
 * sensor (all four steps of sec. 3).  src_dev: float32 [n_src][4] = (x, y, z, weight), weight
 * in [0, 1].  Ray j of source s aims at the aperture point (a sqrt(u1) cos 2 pi u2,
 * a sqrt(u1) sin 2 pi u2) with (u1, u2) the two 24-bit fields of SplitMix64 output number
 * (s << 32 | j) for `seed`.  ds: arc length per Runge-Kutta step (m, > 0).  With stats_host
 * non-NULL the call synchronises the stream and fills the counters; otherwise it is asynchronous.
 * Errors: STATE (field, optics, sensor or trace workspace missing), ARG (n_src < 0, rays_per_src < 1 or
 * >= 2^31, ds <= 0, lens not beyond the box, source array null with n_src > 0),
 * OVERFLOW (n_src * rays_per_src * 2^32 plus what the accumulator may already hold could exceed
 * 2^64 in one pixel), HIP. */
int pbr_emit_and_trace(pbr_ctx *ctx, const float *src_dev, int64_t n_src, int32_t rays_per_src,
                       uint64_t seed, double ds, uint32_t flags, pbr_stats *stats_host);

/* For callers that cannot allocate device memory (code under HIP stream capture, serving loops,
 * harnesses that forbid hipMalloc): pbr_emit_and_trace with the per-ray state of each chunk held
 * in a static device array of the library instead of the context's trace workspace (which need
 * not be set).  Same arguments, flags, results and errors as pbr_emit_and_trace, plus:
 *   rays_per_chunk: rays integrated per launch, in [256, PBR_NOALLOC_MAX_CHUNK] (0 = the maximum);
 *     ARG outside that range.  Images and exit records do not depend on it.
 *   The call allocates no device memory.  Every GPU the library runs on holds one array of
 *   PBR_NOALLOC_MAX_CHUNK x 64 bytes (64 MiB) from its first context until the process ends.
 *   All calls on one GPU share that array: calls whose work overlaps on one GPU (on different
 *   streams, or from different host threads without ordering) race and give wrong results.
 *   With stats_host, box_ms is 0 (no per-launch timing events are created); the other counters
 *   are filled.  With PBR_SURROGATE the attached surrogate must have been created for chunks of
 *   at least rays_per_chunk rays (WORKSPACE otherwise). */
#define PBR_NOALLOC_MAX_CHUNK (1 << 20)
int pbr_emit_and_trace_noalloc(pbr_ctx *ctx, const float *src_dev, int64_t n_src, int32_t rays_per_src,
                               uint64_t seed, double ds, uint32_t flags, int64_t rays_per_chunk,
                               pbr_stats *stats_host);


/* Precision policy for steep-gradient (shock) cells.  Finds the steep bricks of the current field
 * (largest node |grad n| >= steep_frac times the grid maximum), and in each traces rays_per_brick
 * sample rays (uniform start in the brick, aimed at a uniform aperture point) over enough full
 * steps of arc length ds to cross the brick, once in FP32 and once in FP64 from the same state.
 * The difference is measured where it shows: the apparent source point on the focused plane
 * z_focus times |M| / pitch, in pixels.  Bricks whose largest difference exceeds tol_px are flagged;
 * later traces with PBR_PREC_SHOCK_FP64 take their Runge-Kutta steps in FP64 inside flagged bricks
 * and in FP32 elsewhere.  Synchronises the stream.  Uses the trace workspace as scratch.
 * Errors: STATE (field/optics/sensor/trace workspace missing, host-only context), ARG, WORKSPACE. */
int pbr_calibrate_precision(pbr_ctx *ctx, double tol_px, double steep_frac, int32_t rays_per_brick,
                            uint64_t seed, double ds, pbr_precision_report *out);

/* Reads (write = 0) or replaces (write = 1) the per-brick FP64 flags of the current field:
 * n_bricks bytes, brick (bx, by, bz) at (bz * nby + by) * nbx + bx with nb* = ceil((n* - 1) / 8).
 * Synchronises the stream.  Errors: STATE, ARG (n_bricks differs from the grid's). */
int pbr_brick_flags(pbr_ctx *ctx, uint8_t *inout_host, int64_t n_bricks, int write);

/* Converts the accumulator into out_dev (caller-owned: width*height elements of uint64, float
 * or uint16 by fmt).  PBR_FMT_U16 uses `gain` if > 0, else gain = 65535 / (largest pixel value),
 * found on the device.  Errors: ARG, STATE (no sensor). */
int pbr_read_image(pbr_ctx *ctx, int fmt, void *out_dev, double gain);

/* Copies records [first, first + count) of the recording buffer to host memory out_host and
 * synchronises the stream.  Errors: ARG (range outside the buffer), STATE (no recording set). */
int pbr_read_ray_exits(pbr_ctx *ctx, pbr_ray_exit *out_host, int64_t first, int64_t count);

/* ---------------------------------------------------------------- general optical chain (sec. 3.3) */

#define PBR_MAX_SURFACES  16
#define PBR_SURF_REFRACT  0  /* sphere or plane between two media: Snell's law (eq. 7), total internal reflection */
#define PBR_SURF_MIRROR   1  /* reflecting sphere or plane: law of reflection about the local normal */
#define PBR_SURF_APERTURE 2  /* plane stop: rays crossing it farther than `clear` from the axis are blocked */
#define PBR_SURF_LENSLETS 3  /* plane array of spherical lenslets on a square grid of `pitch` centred on the
                                axis (a plenoptic camera's lens array), refracting into n_after; a ray
                                that would meet the cap outside the cell it entered is blocked */

/* One surface, rotationally symmetric about the optical axis (z). */
typedef struct pbr_surface {
    int32_t type;      /* PBR_SURF_* */
    int32_t reserved;
    double z;          /* vertex on the axis (m) */
    double radius;     /* signed radius of curvature (m), centre at z + radius; 0 = plane (ignored for stops) */
    double clear;      /* rays meeting the surface farther than this from the axis are blocked (m), > 0 */
    double n_after;    /* refractive index after the surface (REFRACT, LENSLETS); <= 0 = the ambient index */
    double pitch;      /* LENSLETS: lenslet pitch (m), > 0 */
} pbr_surface;

/* A sequence of surfaces traced in order after the density box (sec. 3.3: mirrors, lenses,
 * windows, apertures and lens arrays), replacing the singlet of pbr_set_optics.  Rays are emitted
 * towards uniform points of the disk of radius aim_radius in the plane z = aim_z (sec. 3.1), then
 * meet each surface at the first intersection ahead of them on the cap around its vertex (a ray
 * that would have to travel backwards is blocked), and finally the sensor plane, which must be
 * given explicitly (pbr_sensor.z_sensor) together with the spot (pbr_sensor.sigma_px > 0): the
 * magnification and f-number of eq. 8 are not defined for a general chain. */
typedef struct pbr_optical_chain {
    int32_t n_surfaces;  /* 1 .. PBR_MAX_SURFACES */
    int32_t reserved;
    double aim_z;        /* plane of the emission target disk, beyond the density box (m) */
    double aim_radius;   /* its radius (m), > 0 */
    pbr_surface s[PBR_MAX_SURFACES];
} pbr_optical_chain;

/* Copies the chain (it may be released on return; the call synchronises the stream) into the
 * context's device block; later traces use it instead of the singlet.  chain = NULL returns to the
 * singlet of pbr_set_optics.  With a chain set, pbr_calibrate_precision, pbr_bos_theory_map,
 * surrogate training and batches (which rely on the singlet's paraxial optics) return STATE.
 * Errors: ARG (bad counts, types, non-finite values, clear <= 0, lenslet pitch <= 0 or a lenslet
 * radius smaller than half the pitch, aim_radius <= 0), HIP. */
int pbr_set_optical_chain(pbr_ctx *ctx, const pbr_optical_chain *chain);

/* ---------------------------------------------------------------- Mie radiance (sec. 3.1) */

/* Angles of the Mie intensity table: theta_k = k pi / (PBR_MIE_TABLE_SIZE - 1). */
#define PBR_MIE_TABLE_SIZE 2049

/* Scattering particles and illumination for ray weights (sec. 3.1: the radiance of a ray depends
 * on the Mie scattering of the particle at the angle between the ray and the laser beam). */
typedef struct pbr_mie {
    double diameter;      /* particle diameter (m), > 0 */
    double m_re, m_im;    /* particle refractive index relative to the ambient medium (m_re > 0, m_im >= 0) */
    double wavelength;    /* laser wavelength in vacuum (m), > 0 */
    double laser_dir[3];  /* propagation direction of the laser light (any length > 0) */
} pbr_mie;

/* The unpolarised Mie intensity (|S1|^2 + |S2|^2) / 2 of the particle at n equally spaced
 * scattering angles over [0, pi], divided by its largest value, for size parameter
 * pi diameter n_medium / wavelength (Bohren & Huffman's series).  Host only, no context.
 * Errors (message in pbr_last_error(NULL)): ARG (null, n < 2, non-finite or out-of-range values,
 * size parameter above 20000). */
int pbr_mie_table(const pbr_mie *mie, double n_medium, double *out_host, int32_t n);

/* Bytes of device memory pbr_set_mie needs: PBR_MIE_TABLE_SIZE doubles. */
size_t pbr_mie_workspace_bytes(void);

/* Computes the intensity table of `mie` in the ambient medium of the current field (n_medium =
 * 1 + K rho_inf) and copies it to table_dev (caller-owned, 8-byte aligned, >=
 * pbr_mie_workspace_bytes, alive while traces use it; the call synchronises the stream).  Traces
 * with PBR_MIE then multiply each ray's source weight by the table at the angle between the ray's
 * direction at its source and the laser direction (linear between nodes), so weights stay in
 * [0, 1].  mie = NULL switches the weighting off.  Errors: ARG, STATE (no field; host-only context
 * after the checks), WORKSPACE, HIP. */
int pbr_set_mie(pbr_ctx *ctx, const pbr_mie *mie, void *table_dev, size_t ws_bytes);

/* ---------------------------------------------------------------- BOS displacement check (sec. 4) */

/* Sums over the deposited rays of one source of their sensor hits (sec. 4 averages the
 * displacements of the rays of each dot).  Fixed point: sum_x = sum of round_half_even(x_px *
 * 2^24) over the rays (likewise y), so the sums are exact integers whatever order the rays
 * arrive in; the mean hit is (sum * 2^-24) / hits. */
typedef struct pbr_source_sum {
    int64_t sum_x;     /* pixels * 2^24, summed */
    int64_t sum_y;
    uint64_t hits;     /* rays of the source deposited on the sensor */
    uint64_t reserved; /* left untouched */
} pbr_source_sum;

/* Order in which a trace with PBR_SOURCE_ORDER takes its sources (sec. 3.5: a source's rays run
 * together and share the cells they cross; neighbouring sources running together share more).
 * order_dev: caller-owned device array of n_src int64 source indices, a permutation of
 * 0 .. n_src - 1, read by every such trace (whose n_src must equal this n_src).  Position q of the
 * processing order is ray q mod rays_per_src of source order_dev[q / rays_per_src], and it keeps
 * that source's key: its random numbers (the SplitMix64 counter of pbr_emit_and_trace), weight,
 * exit-record index and per-source sums are those of the call without an order, so image,
 * records, sums and counters are the same bit for bit; only the order in which rays meet the
 * field, and so the cache reuse between rays in flight together, changes.  An entry outside
 * [0, n_src) is clamped into range (a non-permutation then traces some sources twice and others
 * not at all); the checked build counts such entries and the trace returns PBR_ERR_BOUNDS.  NULL
 * with n_src = 0 clears the order.
 * Errors: ARG (n_src < 0, null with n_src > 0, misaligned). */
int pbr_set_source_order(pbr_ctx *ctx, const int64_t *order_dev, int64_t n_src);

/* Device scratch (bytes) pbr_source_order_morton needs for n_src sources; 0 if n_src < 0 or
 * n_src > 2^31 - 1. */
size_t pbr_source_order_morton_workspace_bytes(int64_t n_src);

/* Writes to order_dev (caller-owned device array of n_src int64) the permutation that sorts the
 * sources of src_dev (float32 [n_src][4] as in pbr_emit_and_trace) by the Morton (Z-order) code of
 * their position in the field's box: 21 bits per axis, positions clamped onto the box, x in the
 * lowest bit; equal codes keep their index order.  Traced in this order, sources that run
 * together lie close together in the field.  Asynchronous on the context's stream.  ws_dev:
 * caller-owned device scratch of at least pbr_source_order_morton_workspace_bytes(n_src) bytes,
 * 256-byte aligned.  Allocates no device memory.
 * Errors: STATE (no field; host-only context), ARG (n_src out of range, null arrays),
 * WORKSPACE, HIP. */
int pbr_source_order_morton(pbr_ctx *ctx, const float *src_dev, int64_t n_src, int64_t *order_dev, void *ws_dev,
                            size_t ws_bytes);

/* Sets the per-source sums that traces with PBR_SOURCE_SUMS add into: sums_dev[s] for source s
 * of the call (caller-owned device array of `capacity` records, 8-byte aligned, which the caller
 * clears; the library only adds).  The traced call must have n_src <= capacity and
 * rays_per_src <= 2^25, which keeps each sum below 2^63 (hits below 16384 pixels).
 * Errors: ARG (null with capacity > 0, capacity < 0, misaligned). */
int pbr_set_source_sums(pbr_ctx *ctx, pbr_source_sum *sums_dev, int64_t capacity);

/* Regular grid of displacement maps on the dot plane: node (i, j) at (x0 + i dx, y0 + j dy,
 * z_dots), 0 <= i < nx, 0 <= j < ny.  Maps are float32 [ny][nx][2] (x and y components). */
typedef struct pbr_map_grid {
    double x0, y0;     /* position of node (0, 0) (m) */
    double dx, dy;     /* node spacing (m), > 0 */
    double z_dots;     /* z of the dot plane (m), in front of the box */
    int32_t nx, ny;    /* nodes, 1 .. 4096 each */
} pbr_map_grid;

/* Workspace bytes of pbr_dot_displacement_map: 24 bytes per node (0 on bad sizes). */
size_t pbr_dot_map_workspace_bytes(int nx, int ny);

/* Map of the per-dot displacements between two renders of the same dots and rays (sec. 4,
 * Fig. 4): with_dev holds the sums of a render through the field, without_dev those of a render
 * through the ambient medium.  Dot s (position src_dev[s].xy) has displacement mean_with -
 * mean_without in pixels when both hit counts are non-zero.  The scattered displacements are
 * placed on the grid by bilinear weights: a dot with fractional cell position (t, u) gives weight
 * (1-t)(1-u), t(1-u), (1-t)u, tu to the four nodes around it; a node's value is the weighted mean
 * of what it received (weights and weighted displacements summed as integers in units of 2^-32,
 * rounded half to even), NaN where nothing arrived.  ws_dev: pbr_dot_map_workspace_bytes,
 * 8-byte aligned, scratch.  map_dev: float32 [ny][nx][2].  Asynchronous.
 * Errors: ARG (null pointers, bad grid, n_src < 0), WORKSPACE, STATE (host-only context), HIP. */
int pbr_dot_displacement_map(pbr_ctx *ctx, const pbr_source_sum *with_dev,
                             const pbr_source_sum *without_dev, const float *src_dev, int64_t n_src,
                             const pbr_map_grid *grid, void *ws_dev, size_t ws_bytes, float *map_dev);

/* Eq. 9 at the grid nodes: the displacement, in pixels, that BOS theory predicts for a dot at the
 * node, |M| Z_D / n0 times the integral over the box depth of (dn/dx, dn/dy) dz along the chief
 * ray from the node to the centre of the aperture stop; M is the paraxial magnification of the
 * dot plane, Z_D the distance from the dot plane to the mid-plane of the box, n0 the ambient
 * index.  The integral is the midpoint rule with `samples` points over the box's z extent, the
 * gradient interpolated from the current field; points outside the box's x-y extent add nothing.
 * The sign is that of the unflipped sensor.  map_dev: float32 [ny][nx][2].  Needs field, optics
 * and sensor.  Asynchronous.  Errors: ARG (bad grid, samples < 1 or > 65536, dot plane not in
 * front of the box), STATE, HIP. */
int pbr_bos_theory_map(pbr_ctx *ctx, const pbr_map_grid *grid, int32_t samples, float *map_dev);

/* ---------------------------------------------------------------- PIV frame pairs (sec. 1) */

/* Second frame of a PIV pair (sec. 1: velocity is measured from the displacement of the particles
 * between two frames).  Advances every particle of src_in_dev (float32 [n_src][4] = x, y, z, weight)
 * by dx/dt = u(x) over dt (s) with `substeps` classical fourth-order Runge-Kutta steps in FP64 and
 * writes (x', y', z', weight) to src_out_dev (which may be src_in_dev).  vel_dev: float32
 * [nz][ny][nx][3] velocity (u, v, w in m/s) at nodes origin + (i, j, k) * spacing, interpolated
 * trilinearly; a point outside the grid takes the value at the nearest point of the grid.
 * Rendering both frames with the same seed gives every ray of a particle the same aperture point
 * in both, so the pair differs only by the motion.  Asynchronous.
 * Errors: ARG (null or misaligned arrays: sources 16 bytes, velocity 4; n_src < 0; dims < 2 or
 * > 65535 or more than 2^31 nodes; spacing <= 0 or non-finite; non-finite origin or dt; substeps
 * outside 1 .. 4096), STATE (host-only context), HIP. */
int pbr_displace_sources(pbr_ctx *ctx, const float *src_in_dev, float *src_out_dev, int64_t n_src,
                         const float *vel_dev, int nx, int ny, int nz, const double origin[3],
                         const double spacing[3], double dt, int32_t substeps);

/* ---------------------------------------------------------------- batches of images */

/* Many images (each its own context: field, optics, sensor, accumulator, exit recording, all set
 * beforehand on one GPU) traced in one graph-captured launch sequence.  The batch snapshots each
 * context's field, optics, sensor and recording at pbr_batch_create.  Image k of a batch is bit
 * for bit the image pbr_emit_and_trace would render alone (integer deposits, same per-ray
 * arithmetic).  Integration is FP32.
 *
 * The rays of all images are laid out in rounds (at most round_rays ray states each): images in
 * decreasing estimated cost per ray (box depth / ds), each split across rounds as needed and
 * padded to whole blocks of 256 rays.  A round is three kernels: emission, a persistent
 * integration kernel in which every wave pulls the next unit_rays rays from a global counter, and
 * lens / sensor / deposit (LDS tile of tile x tile pixels).  The first pbr_batch_run after
 * creation or pbr_batch_configure captures clears, counters and all rounds into one HIP graph;
 * later runs replay it. */
typedef struct pbr_batch pbr_batch;

typedef struct pbr_batch_item {
    pbr_ctx *ctx;            /* the image's context */
    const float *src_dev;    /* float32 [n_src][4] sources, 16-byte aligned (as pbr_emit_and_trace) */
    int64_t n_src;
    int32_t rays_per_src;
    uint32_t flags;          /* PBR_CLEAR_FIRST and/or PBR_RECORD_EXITS only */
    uint64_t seed;
    double ds;
} pbr_batch_item;

typedef struct pbr_batch_config {
    int32_t box_block;       /* threads per block of the persistent integration kernel: 64 or 256 */
    int32_t unit_rays;       /* rays a wave pulls from the work queue at a time: 64, 128 or 256 */
    int32_t tile;            /* deposit pre-aggregation tile side in pixels: 16 or 32 */
    int32_t reserved;
    int64_t round_rays;      /* ray states per round, multiple of 256 in [min_round_rays, max_round_rays] */
    int64_t max_round_rays;  /* (out) the largest round the workspace holds */
    int64_t min_round_rays;  /* (out) the smallest round the segment table allows */
    int32_t rounds;          /* (out) rounds of the current plan */
    int32_t pad;
} pbr_batch_config;

typedef struct pbr_batch_stats {
    uint64_t rays;
    uint64_t status[PBR_NUM_STATUS];
    uint64_t rkn_steps;
    double run_ms;           /* device time of the graph launch (HIP events) */
    int32_t rounds;
    int32_t images;
    uint64_t rkn_steps_nodes; /* of rkn_steps, those of images with a node-layout field */
} pbr_batch_stats;

/* Workspace bytes for a batch whose rounds hold up to round_rays rays (64 bytes per ray state
 * plus parameters and segment tables); 0 on bad arguments. */
size_t pbr_batch_workspace_bytes(const pbr_batch_item *items, int n_items, int64_t round_rays);

/* Validates every item (as pbr_emit_and_trace would), uploads per-image launch parameters into
 * ws_dev (256-byte aligned, caller-owned, live until pbr_batch_destroy) and plans the rounds with
 * the default configuration (box_block 64, unit_rays 64, tile 32, largest round).  Launches and
 * graph replays go to hip_stream.  Errors: ARG, STATE (a context lacks field/optics/sensor),
 * WORKSPACE, OVERFLOW, HIP; the message is in pbr_batch_last_error(NULL). */
int pbr_batch_create(pbr_batch **out, const pbr_batch_item *items, int n_items, void *ws_dev,
                     size_t ws_bytes, void *hip_stream);
void pbr_batch_destroy(pbr_batch *b);
const char *pbr_batch_last_error(const pbr_batch *b);
int pbr_batch_get_config(pbr_batch *b, pbr_batch_config *out);
/* Re-plans with a new configuration (drops the captured graph).  Errors: ARG. */
int pbr_batch_configure(pbr_batch *b, const pbr_batch_config *cfg);
/* Runs the whole batch (graph launch); with stats non-NULL synchronises and sums the counters of
 * all images.  Errors: OVERFLOW (an accumulating item would exceed 2^32 - 1 rays), HIP. */
int pbr_batch_run(pbr_batch *b, pbr_batch_stats *stats);
/* Autotuner of the batched launch.  With cache_path naming a file that holds a choice for this
 * device and batch shape (architecture, grid and sensor sizes, field layout, source and ray counts
 * of every image), that choice is applied.  Otherwise every combination of box_block {64, 256},
 * unit_rays {64, 256}, tile {16, 32} and round_rays {largest, half} is timed on the first
 * probe_rounds rounds (direct launches, HIP events; median of three passes after a warm-up), the
 * three fastest are timed again (median of five) and the fastest of those (rays per ms) is applied
 * and appended to cache_path (if given).  Leaves the accumulators and counters of the batch's images
 * in an unspecified state: run the batch with PBR_CLEAR_FIRST items afterwards.  Synchronises. */
int pbr_batch_autotune(pbr_batch *b, const char *cache_path, int32_t probe_rounds, pbr_batch_config *chosen,
                       double *rays_per_ms);

/* ---------------------------------------------------------------- ray surrogate network
 * A multilayer perceptron 6 -> 256 -> 256 -> 256 -> 256 -> 6 with GELU activations (tanh form,
 * Hendrycks & Gimpel 2016) that stands in for the integration of the ray equation (eqs. 3-6)
 * through one fixed density field: from a ray's entry through the box face z = z_min it predicts
 * where, and in which direction, the ray leaves through the face z = z_max.  Everything before
 * (emission) and after (lens, eq. 7; deposit, eq. 8) stays the tracer's.
 *
 * Inputs (features): entry x and y scaled to [-1, 1] over the box, the entry direction's x and y
 * components over their RMS theta in the training set, sin(2 pi (x - x_min) / L_x) and
 * sin(2 pi (y - y_min) / L_y).  Outputs: exit position minus the straight-line exit from the same
 * entry (x, y, z; z is always 0) and exit unit direction minus entry unit direction, each
 * standardised with the training set's mean and standard deviation.
 *
 * Parameters are FP32 in one flat array of PBR_SURR_PARAMS floats: W1 [256][6], b1 [256],
 * W2 [256][256], b2, W3, b3, W4, b4, W5 [6][256], b5 [6] (row-major, W[out][in]).  Matrix products
 * of layers 2-5 run on bfloat16 copies of the weights and activations with FP32 accumulation;
 * layer 1 and all pre-activations, biases and gradient sums stay FP32.  Training: mean squared
 * error over the standardised outputs, Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master
 * weights.
 *
 * A trained surrogate belongs to the context it was trained on, and only while that context's
 * field, optics and sensor stay as they were.  Its fallback map splits the entry face into
 * tiles x tiles tiles: a tile is eligible only when every validation ray entering through it
 * lands within tol_px (sensor pixels) of where the tracer puts it; all other rays are traced. */
#define PBR_SURR_PARAMS 200710

typedef struct pbr_surrogate pbr_surrogate;

typedef struct pbr_surrogate_train_config {
    int32_t batch;             /* rows per Adam step, a multiple of 64 not above max_rows */
    int32_t epochs;            /* passes over the training rays */
    float lr_max, lr_min;      /* learning rate: cosine from lr_max (first step) to lr_min (last) */
    double tol_px;             /* eligibility tolerance on the sensor, pixels (0.01) */
    int32_t tiles;             /* tiles per side of the entry face, 1 .. 1024 */
    int32_t min_tile_samples;  /* tiles with fewer validation rays stay ineligible (>= 1) */
    uint64_t shuffle_seed;     /* order of the training rays in each epoch */
} pbr_surrogate_train_config;

typedef struct pbr_surrogate_report {
    int64_t train_samples;     /* training rays that cross the box from face z_min to face z_max */
    int64_t val_samples;       /* validation rays that cross and reach the sensor */
    int64_t val_eligible;      /* of which enter through eligible tiles */
    int64_t val_rim_mismatches; /* validation rays that reach the sensor either from the tracer's or
                                   from the predicted exit but not both (aperture or lens rim) */
    int32_t steps;             /* Adam steps taken */
    int32_t eligible_tiles;
    double loss_first_epoch;   /* mean training loss over the first and the last epoch */
    double loss_last_epoch;
    double val_median_px;      /* sensor-hit error over all validation samples */
    double val_p99_px;
    double val_max_px;
    double val_max_eligible_px;
    double sample_ms;          /* wall time of tracing the training and validation rays */
    double train_ms;           /* wall time of the Adam steps */
    double validate_ms;
} pbr_surrogate_report;

/* Device bytes of a surrogate's persistent workspace: FP32 parameters, gradient and Adam moments,
 * bfloat16 weight copies, training-pass buffers for max_rows rows (rounded up to 64; 65536 if 0),
 * inference buffers for trace chunks of up to ray_chunk rays (53 bytes per ray; 0 when the
 * surrogate never runs inside a trace) and a 1 MiB tile map.  0 for arguments out of range
 * (max_rows in [0, 2^24], ray_chunk in [0, 2^31]). */
size_t pbr_surrogate_workspace_bytes(int64_t max_rows, int64_t ray_chunk);

/* Creates a network on device (current device if -1) with weights and biases drawn uniformly from
 * +-1/sqrt(fan_in) (SplitMix64 of init_seed) and zero Adam moments, all held in the caller's
 * workspace ws_dev (device, 256-byte aligned, at least pbr_surrogate_workspace_bytes(max_rows,
 * ray_chunk) bytes, alive and untouched until pbr_surrogate_destroy).  Traces with PBR_SURROGATE
 * on contexts whose chunk exceeds ray_chunk fail with WORKSPACE.  hip_stream: stream for the
 * calls below (NULL = the null stream); training and the trace hook enqueue on the context's
 * stream instead.  Allocates no device memory.
 * Errors: ARG, WORKSPACE, HIP (see pbr_surrogate_last_error(NULL) when *out is NULL). */
int pbr_surrogate_create(pbr_surrogate **out, int device, void *hip_stream, uint64_t init_seed, int64_t max_rows,
                         int64_t ray_chunk, void *ws_dev, size_t ws_bytes);
void pbr_surrogate_destroy(pbr_surrogate *s);
const char *pbr_surrogate_last_error(const pbr_surrogate *s);

/* Copies all PBR_SURR_PARAMS parameters from / to host memory (n must equal PBR_SURR_PARAMS);
 * set also resets the Adam moments.  Synchronises.  Errors: ARG, HIP. */
int pbr_surrogate_set_params(pbr_surrogate *s, const float *params_host, int64_t n);
int pbr_surrogate_get_params(pbr_surrogate *s, float *params_host, int64_t n);

/* Network outputs for rows inputs: x_dev [rows][6] -> y_dev [rows][6], device memory, FP32.
 * Enqueued on the surrogate's stream.  Errors: ARG, HIP. */
int pbr_surrogate_forward(pbr_surrogate *s, const float *x_dev, int64_t rows, float *y_dev);

/* Mean squared error of the outputs for x_dev against targets t_dev (both [rows][6], device) and
 * its gradient with respect to every parameter (grad_host: PBR_SURR_PARAMS floats, may be NULL).
 * rows: a positive multiple of 64 not above max_rows.  Synchronises.  Errors: ARG, HIP. */
int pbr_surrogate_gradients(pbr_surrogate *s, const float *x_dev, const float *t_dev, int64_t rows,
                            float *grad_host, double *loss_host);

/* One Adam step (step = 1, 2, ... as in the bias corrections) on the gradient of x_dev, t_dev as
 * above, learning rate lr.  loss_host (may be NULL) receives the loss before the step.
 * Synchronises only when loss_host is given.  Errors: ARG, HIP. */
int pbr_surrogate_adam_step(pbr_surrogate *s, const float *x_dev, const float *t_dev, int64_t rows, float lr,
                            int32_t step, double *loss_host);

/* Trains the network for the context's current field, optics and sensor.  The tracer (FP32; FP64
 * inside flagged bricks when the context has any) integrates n_train_src x train_rays_per_src rays
 * emitted from train_src_dev with train_seed, and n_val_src x val_rays_per_src from val_src_dev
 * with val_seed (device arrays as in pbr_emit_and_trace), without depositing them.  (The rays of
 * one source enter the box close together: many sources with few rays each cover more tiles.)  Rays that enter
 * through z_min and leave through z_max become samples; the training samples set the
 * standardisation, then cfg->epochs passes of Adam steps over shuffled batches of cfg->batch;
 * the validation samples that reach the sensor are pushed through lens and sensor from the
 * predicted exit and compared with the tracer's hit, which fixes the fallback map (a tile with a
 * validation ray that enters through z_min but leaves through another face is never eligible;
 * rays that reach the sensor one way but not the other are counted and make their tile
 * ineligible too).  The
 * context's sensor accumulator and counters are left untouched; its trace workspace is used as
 * scratch.  ws_dev: training scratch (device, 256-byte aligned, at least
 * pbr_surrogate_train_workspace_bytes bytes for these ray counts and cfg; free again when the
 * call returns): the samples (88 bytes per ray), shuffles, losses and validation errors.
 * Allocates no device memory.  Synchronises.
 * Errors: STATE (context not ready, host-only context), ARG, WORKSPACE, HIP. */
size_t pbr_surrogate_train_workspace_bytes(int64_t n_train_rays, int64_t n_val_rays, int32_t batch, int32_t epochs,
                                           int32_t tiles);
int pbr_surrogate_train(pbr_surrogate *s, pbr_ctx *ctx, const float *train_src_dev, int64_t n_train_src,
                        int32_t train_rays_per_src, const float *val_src_dev, int64_t n_val_src,
                        int32_t val_rays_per_src, uint64_t train_seed, uint64_t val_seed, double ds,
                        const pbr_surrogate_train_config *cfg, void *ws_dev, size_t ws_bytes,
                        pbr_surrogate_report *report);

/* Fallback map of a trained surrogate: tiles x tiles bytes (1 = eligible) and the largest
 * validation error per tile in pixels (-1 for tiles without validation rays), tile (tx, ty) at
 * ty * tiles + tx, tx along x.  Either pointer may be NULL.  Errors: STATE (not trained), ARG. */
int pbr_surrogate_tile_map(pbr_surrogate *s, uint8_t *eligible_host, float *max_err_host, int64_t n_tiles);

/* Persisting a trained surrogate (weights, Adam state, input/output scaling, tile map) as a
 * self-checking host blob.  pbr_surrogate_blob_bytes: its size (0 unless trained).
 * pbr_surrogate_save writes it (synchronises; errors: STATE untrained, WORKSPACE cap too small, HIP).
 * pbr_surrogate_load restores it into `s` and binds it to `ctx`, which must hold the scene it was
 * trained on: the same stored field (geometry and a device checksum of the field), optics, sensor
 * and optical chain; traces must use the training step length ds.  Errors: ARG (not a blob,
 * damaged, another version or network), STATE (the scene differs, host-only context), HIP. */
size_t pbr_surrogate_blob_bytes(pbr_surrogate *s);
int pbr_surrogate_save(pbr_surrogate *s, void *buf_host, size_t cap);
int pbr_surrogate_load(pbr_surrogate *s, pbr_ctx *ctx, const void *buf_host, size_t size);

/* Attaches a trained surrogate to the context it was trained on (NULL detaches).  Traces with
 * PBR_SURROGATE then hand every ray that enters through an eligible tile of z_min to the network
 * and trace the rest.  Fails with STATE when the surrogate is untrained, was trained on another
 * context or the context's field, optics or sensor changed since.  The surrogate must outlive
 * the attachment. */
int pbr_set_surrogate(pbr_ctx *ctx, pbr_surrogate *s);

/* ---------------------------------------------------------------- calibration probe
 * Rate of 64-bit integer atomic additions the device sustains: n_updates additions spread over
 * n_slots 8-byte counters (groups of 256 consecutive updates hit consecutive counters, as the
 * pixels of a spot do), timed with HIP events on the null stream after one warm-up launch.
 * Allocates and frees its own buffer; synchronises.  Errors: ARG, HIP. */
int pbr_probe_u64_atomics(int device, int64_t n_slots, int64_t n_updates, double *updates_per_s);

/* Vector fused multiply-add rate of the device in FLOP/s (2 per FMA): FP32 (fp64 = 0; plain
 * single-lane instructions, the library being built with packed FP32 instructions disabled) or
 * FP64, eight independent chains per lane, four 256-thread blocks per SIMD, timed as above after
 * a warm-up launch.  The ceiling of the integration kernels' arithmetic.  Allocates and frees its own
 * output buffer; synchronises.  Errors: ARG, HIP. */
int pbr_probe_fma_rate(int device, int fp64, double *flop_per_s);

/* Read bandwidth in bytes/s: total_bytes read as float4 from a buffer of buffer_bytes (a power of
 * two, >= 64 KiB, zero-filled; read repeatedly when smaller than total_bytes).  A buffer that fits
 * the L2 caches (a few MiB) measures L2 bandwidth, one far above the 256 MB Infinity Cache measures
 * HBM.  scattered = 0: consecutive lanes read consecutive 16-byte words (fully used lines);
 * scattered = 1: every lane reads one 16-byte word of its own 128-byte line (the shape of a field
 * gather whose lanes sit in different cells).  Allocates and frees its buffers; synchronises.
 * Errors: ARG (sizes), HIP. */
int pbr_probe_read_bandwidth(int device, int64_t buffer_bytes, int64_t total_bytes, int scattered,
                             double *bytes_per_s);

/* LDS read bandwidth in bytes/s (16-byte reads without bank conflicts, four 256-thread blocks per
 * SIMD).  Synchronises.  Errors: ARG, HIP. */
int pbr_probe_lds_bandwidth(int device, double *bytes_per_s);

#ifdef __cplusplus
}
#endif

#endif /* PBR_H */
