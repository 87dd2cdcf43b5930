// Internal structures shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pbr.h"

namespace pbr {

// Counter block layout (uint64 slots in the context's device block).
enum : int {
    CNT_STATUS = 0,                       // PBR_NUM_STATUS slots
    CNT_ENTERED = PBR_NUM_STATUS,         // rays that entered the box
    CNT_STEPS = PBR_NUM_STATUS + 1,       // Runge-Kutta steps
    CNT_MAXPIX = PBR_NUM_STATUS + 2,      // largest accumulator value (readout)
    CNT_SLOTS = 16
};

constexpr int kMaxFootprint = 8;          // deposit window half-width limit (sigma <= 2.67 px)

// Everything one trace launch reads.  Passed by value as the kernel argument.
struct TraceParams {
    // field: float4 (n - 1, dn/dx, dn/dy, dn/dz) per node, [nz][ny][nx]
    const float4 *node;
    int nx, ny, nz;
    int max_steps;
    double origin[3], spacing[3];
    double lo[3], hi[3];
    double step_cell[3];   // h / spacing: cell units moved per unit of T in one full step
    double h;              // step of the ray parameter t (dR/dt = T): ds / n_inf
    double n_inf;
    // sources and rays
    const float4 *src;
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
    int pad0;
    // exit records
    pbr_ray_exit *rec;
    int64_t rec_first, rec_stride, rec_max;
    // counters
    unsigned long long *counters;
};

// Launchers (defined in the .hip files; enqueue on `stream`, return hipError_t as int).
int launch_field_prep(const float *rho, float4 *node, int nx, int ny, int nz,
                      const double spacing[3], double K, hipStream_t stream);
int launch_trace(const TraceParams &p, bool fp64, hipStream_t stream);
int launch_readout(const unsigned long long *accum, int64_t npx, int fmt, void *out,
                   double gain, unsigned long long *counters, hipStream_t stream);
int launch_clear_u64(unsigned long long *p, int64_t n, hipStream_t stream);

}  // namespace pbr
