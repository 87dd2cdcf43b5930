// The BOS displacement check of sec. 4 (Fig. 4, eq. 9): the per-dot displacements between a
// render through the field and one through the ambient medium, placed on a regular grid by
// bilinear weights, and the displacement eq. 9 predicts at the grid nodes.  Both are small next to
// the two renders (one thread per dot, one wave per eq. 9 node).
#include "pbr_internal.h"

namespace pbr {
namespace {

constexpr double kQ24 = 16777216.0;
constexpr double kQ32 = 4294967296.0;

__device__ __forceinline__ void add_u64(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256) k_map_clear(unsigned long long *ws, int64_t n)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        ws[k] = 0ull;
}

// Mean hit of a source from its sums: (sum * 2^-24) / hits.
__device__ __forceinline__ double mean_hit(int64_t sum, uint64_t hits)
{
    #pragma clang fp contract(off)
    return ((double)sum / kQ24) / (double)hits;
}

// One dot: its displacement (pixels) spread over the four nodes around it with bilinear weights,
// summed as integers in units of 2^-32 (per node: weight, weight * dx, weight * dy).
__global__ void __launch_bounds__(256) k_dot_splat(const pbr_source_sum *__restrict__ with_sums,
                                                   const pbr_source_sum *__restrict__ without_sums,
                                                   const float4 *__restrict__ src, int64_t n, pbr_map_grid g,
                                                   unsigned long long *__restrict__ ws)
{
    #pragma clang fp contract(off)
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const pbr_source_sum a = with_sums[s], b = without_sums[s];
    if (a.hits == 0 || b.hits == 0) return;
    const double ddx = mean_hit(a.sum_x, a.hits) - mean_hit(b.sum_x, b.hits);
    const double ddy = mean_hit(a.sum_y, a.hits) - mean_hit(b.sum_y, b.hits);
    const float4 p = src[s];
    const double fx = ((double)p.x - g.x0) / g.dx;
    const double fy = ((double)p.y - g.y0) / g.dy;
    if (!(fx > -1.0 && fy > -1.0 && fx < (double)g.nx && fy < (double)g.ny)) return;
    const double ox = floor(fx), oy = floor(fy);
    const int i = (int)ox, j = (int)oy;
    const double t = fx - ox, u = fy - oy;
    const double w[4] = {(1.0 - t) * (1.0 - u), t * (1.0 - u), (1.0 - t) * u, t * u};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int ii = i + (k & 1), jj = j + (k >> 1);
        if (ii < 0 || jj < 0 || ii >= g.nx || jj >= g.ny) continue;
        unsigned long long *node = ws + 3 * ((size_t)jj * (size_t)g.nx + (size_t)ii);
        add_u64(node, (unsigned long long)(long long)rint(w[k] * kQ32));
        add_u64(node + 1, (unsigned long long)(long long)rint((w[k] * ddx) * kQ32));
        add_u64(node + 2, (unsigned long long)(long long)rint((w[k] * ddy) * kQ32));
    }
}

__global__ void __launch_bounds__(256) k_map_finish(const unsigned long long *__restrict__ ws, int64_t n_nodes,
                                                    float *__restrict__ map)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n_nodes) return;
    const unsigned long long w = ws[3 * k];
    float vx = __builtin_nanf(""), vy = __builtin_nanf("");
    if (w) {
        vx = (float)((double)(long long)ws[3 * k + 1] / (double)w);
        vy = (float)((double)(long long)ws[3 * k + 2] / (double)w);
    }
    map[2 * k] = vx;
    map[2 * k + 1] = vy;
}

// (dn/dx, dn/dy) at a point inside the box from the trilinear coefficients of its cell.
__device__ __forceinline__ void grad_xy(const TraceParams &P, const double R[3], double *gx, double *gy)
{
    #pragma clang fp contract(off)
    const int n3[3] = {P.nx, P.ny, P.nz};
    int c[3];
    double w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double f = (R[a] - P.origin[a]) / P.spacing[a];
        f = fmin(fmax(f, 0.0), (double)(n3[a] - 1));
        int i = (int)floor(f);
        i = min(i, n3[a] - 2);
        c[a] = i;
        w[a] = f - (double)i;
    }
    float4 k[kCellFloat4];
    if (P.node_layout) {  // corners (n - 1, grad n) -> the coefficients of the cell records
        const size_t sy = (size_t)P.nx, sz = (size_t)P.nx * (size_t)P.ny;
        const float4 *b = P.cells + (size_t)c[2] * sz + (size_t)c[1] * sy + (size_t)c[0];
        const float4 v000 = b[0], v100 = b[1], v010 = b[sy], v110 = b[sy + 1];
        const float4 v001 = b[sz], v101 = b[sz + 1], v011 = b[sz + sy], v111 = b[sz + sy + 1];
        k[0] = v000;
        k[1] = v100 - v000;
        k[2] = v010 - v000;
        k[3] = v001 - v000;
        k[4] = (v110 - v010) - k[1];
        k[5] = (v101 - v001) - k[1];
        k[6] = (v011 - v001) - k[2];
        k[7] = (((v111 - v011) - (v110 - v010)) - (v101 - v001)) + k[1];
    } else {
        const float4 *q =
            P.cells + ((size_t)(c[2] * (P.ny - 1) + c[1]) * (size_t)(P.nx - 1) + (size_t)c[0]) * kCellFloat4;
#pragma unroll
        for (int m = 0; m < kCellFloat4; ++m) k[m] = q[m];
    }
    const double x = w[0], y = w[1], z = w[2];
    // v = c0 + z c3 + y (c2 + z c6) + x (c1 + y (c4 + z c7) + z c5)
    *gx = (double)k[0].y + z * (double)k[3].y + y * ((double)k[2].y + z * (double)k[6].y) +
          x * ((double)k[1].y + y * ((double)k[4].y + z * (double)k[7].y) + z * (double)k[5].y);
    *gy = (double)k[0].z + z * (double)k[3].z + y * ((double)k[2].z + z * (double)k[6].z) +
          x * ((double)k[1].z + y * ((double)k[4].z + z * (double)k[7].z) + z * (double)k[5].z);
}

// Eq. 9 at one node per wave: midpoint rule along the chief ray from the node to the aperture
// centre, lane l taking samples l, l + 64, ...; the partial sums are then added across the wave.
__global__ void __launch_bounds__(256) k_bos_theory(TraceParams P, pbr_map_grid g, double scale, int samples,
                                                    float *__restrict__ map)
{
    #pragma clang fp contract(off)
    const int64_t node = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
    if (node >= (int64_t)g.nx * g.ny) return;  // whole waves
    const int lane = (int)(threadIdx.x & 63u);
    const int i = (int)(node % g.nx), j = (int)(node / g.nx);
    const double X = g.x0 + (double)i * g.dx, Y = g.y0 + (double)j * g.dy;
    const double dz = (P.hi[2] - P.lo[2]) / (double)samples;
    double sx = 0.0, sy = 0.0;
    for (int k = lane; k < samples; k += 64) {
        const double z = P.lo[2] + ((double)k + 0.5) * dz;
        const double f = (z - g.z_dots) / (P.z_lens - g.z_dots);
        const double R[3] = {X * (1.0 - f), Y * (1.0 - f), z};
        if (R[0] < P.lo[0] || R[0] > P.hi[0] || R[1] < P.lo[1] || R[1] > P.hi[1]) continue;
        double gx, gy;
        grad_xy(P, R, &gx, &gy);
        sx += gx;
        sy += gy;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
    }
    if (lane == 0) {
        map[2 * node] = (float)(scale * sx * dz);
        map[2 * node + 1] = (float)(scale * sy * dz);
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int launch_dot_map(const pbr_source_sum *with_sums, const pbr_source_sum *without_sums, const float4 *src,
                   int64_t n_src, const pbr_map_grid &g, unsigned long long *ws, float *map, hipStream_t stream)
{
    const int64_t nodes = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL(k_map_clear, dim3(blocks_for(3 * nodes) < 4096u ? blocks_for(3 * nodes) : 4096u), dim3(256),
                       0, stream, ws, 3 * nodes);
    if (n_src > 0)
        hipLaunchKernelGGL(k_dot_splat, dim3(blocks_for(n_src)), dim3(256), 0, stream, with_sums, without_sums,
                           src, n_src, g, ws);
    hipLaunchKernelGGL(k_map_finish, dim3(blocks_for(nodes)), dim3(256), 0, stream, ws, nodes, map);
    return (int)hipGetLastError();
}

int launch_bos_theory(const TraceParams &p, const pbr_map_grid &g, double scale, int samples, float *map,
                      hipStream_t stream)
{
    const int64_t nodes = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL(k_bos_theory, dim3((unsigned)((nodes + 3) / 4)), dim3(256), 0, stream, p, g, scale, samples,
                       map);
    return (int)hipGetLastError();
}

}  // namespace pbr
