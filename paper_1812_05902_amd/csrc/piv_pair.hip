// Second frame of a PIV pair (sec. 1: the velocity is measured from the displacement of the
// particles between two frames): every particle advanced by a prescribed velocity field over the
// frame interval.  One thread per particle; the cost is negligible next to rendering a frame.
#include "piv_internal.h"

namespace pbr {
namespace {

// Velocity at x: trilinear in the cell holding the point (a point outside the grid is first moved
// onto it), from float32 nodes vel[(k ny + j) nx + i][3].
__device__ __forceinline__ void vel_at(const VelocityGrid &g, const double x[3], double u[3])
{
    #pragma clang fp contract(off)
    const int n3[3] = {g.nx, g.ny, g.nz};
    int c[3];
    double w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double f = (x[a] - g.origin[a]) / g.spacing[a];
        f = fmin(fmax(f, 0.0), (double)(n3[a] - 1));
        int i = (int)floor(f);
        i = min(i, n3[a] - 2);
        c[a] = i;
        w[a] = f - (double)i;
    }
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                const double wt = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
                const float *p = g.vel + 3 * (((size_t)(c[2] + dk) * (size_t)g.ny + (size_t)(c[1] + dj)) *
                                                  (size_t)g.nx + (size_t)(c[0] + di));
#pragma unroll
                for (int q = 0; q < 3; ++q) v[q] += wt * (double)p[q];
            }
    u[0] = v[0];
    u[1] = v[1];
    u[2] = v[2];
}

// dx/dt = u(x) over dt by `substeps` classical fourth-order Runge-Kutta steps, in FP64.
__global__ void __launch_bounds__(256) k_displace(const float4 *__restrict__ in, float4 *__restrict__ out,
                                                  int64_t n, VelocityGrid g, double dt, int substeps)
{
    #pragma clang fp contract(off)
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float4 p = in[s];
    double x[3] = {(double)p.x, (double)p.y, (double)p.z};
    const double h = dt / (double)substeps;
    for (int m = 0; m < substeps; ++m) {
        double k1[3], k2[3], k3[3], k4[3], q[3];
        vel_at(g, x, k1);
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = x[a] + 0.5 * h * k1[a];
        vel_at(g, q, k2);
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = x[a] + 0.5 * h * k2[a];
        vel_at(g, q, k3);
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = x[a] + h * k3[a];
        vel_at(g, q, k4);
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] += h * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]) / 6.0;
    }
    out[s] = make_float4((float)x[0], (float)x[1], (float)x[2], p.w);
}

}  // namespace

int launch_displace(const float4 *in, float4 *out, int64_t n, const VelocityGrid &g, double dt, int substeps,
                    hipStream_t stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_displace, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, in, out, n, g, dt,
                       substeps);
    return (int)hipGetLastError();
}

}  // namespace pbr
