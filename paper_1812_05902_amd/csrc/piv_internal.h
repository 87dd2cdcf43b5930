// PIV frame pairs: the displacement kernel's launch interface (piv_pair.hip).
#pragma once
#include "pbr_internal.h"

namespace pbr {

// Prescribed velocity on a node grid, float32 [nz][ny][nx][3] (u, v, w).
struct VelocityGrid {
    const float *vel;
    int nx, ny, nz;
    double origin[3], spacing[3];
};

// src_out[s] = src_in[s] advanced by the velocity over dt (substeps RK4 steps), weight copied.
int launch_displace(const float4 *in, float4 *out, int64_t n, const VelocityGrid &g, double dt, int substeps,
                    hipStream_t stream);

}  // namespace pbr
