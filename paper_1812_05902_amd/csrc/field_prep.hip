// Field preparation (sec. 3.2): Gladstone-Dale n = K rho + 1 (eq. 1) and the refractive-index
// gradient at every grid node, written as one float4 (n - 1, dn/dx, dn/dy, dn/dz) per node.
//
// The arithmetic is FP64 (the inputs are float32 densities, the outputs are rounded once to
// float32), so the stored values are the exact node values to float32 rounding.  The kernel is
// bound by HBM: 4 B read (plus cached neighbour reads) and 16 B written per node.
#include "pbr_internal.h"

namespace pbr {
namespace {

// Derivative with respect to the node index along one grid line: central difference inside,
// second-order one-sided difference on the first and last node, plain difference when the line
// has only two nodes.
__device__ __forceinline__ double index_derivative(const float *__restrict__ rho, size_t q,
                                                   size_t stride, int m, int n)
{
    if (n == 2) {
        const size_t q0 = q - (size_t)m * stride;
        return (double)rho[q0 + stride] - (double)rho[q0];
    }
    if (m == 0)
        return -1.5 * (double)rho[q] + 2.0 * (double)rho[q + stride] - 0.5 * (double)rho[q + 2 * stride];
    if (m == n - 1)
        return 1.5 * (double)rho[q] - 2.0 * (double)rho[q - stride] + 0.5 * (double)rho[q - 2 * stride];
    return 0.5 * ((double)rho[q + stride] - (double)rho[q - stride]);
}

__global__ void __launch_bounds__(256)
k_field_prep(const float *__restrict__ rho, float4 *__restrict__ node, int nx, int ny, int nz,
             double kx, double ky, double kz, double K)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= nx) return;
    const size_t sx = 1, sy = (size_t)nx, sz = (size_t)nx * (size_t)ny;
    const size_t q = (size_t)k * sz + (size_t)j * sy + (size_t)i;
    float4 out;
    out.x = (float)(K * (double)rho[q]);
    out.y = (float)(kx * index_derivative(rho, q, sx, i, nx));
    out.z = (float)(ky * index_derivative(rho, q, sy, j, ny));
    out.w = (float)(kz * index_derivative(rho, q, sz, k, nz));
    node[q] = out;
}

__global__ void __launch_bounds__(256) k_clear_u64(unsigned long long *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = 0ull;
}

}  // namespace

int launch_field_prep(const float *rho, float4 *node, int nx, int ny, int nz,
                      const double spacing[3], double K, hipStream_t stream)
{
    dim3 block(256);
    dim3 grid((unsigned)((nx + 255) / 256), (unsigned)ny, (unsigned)nz);
    hipLaunchKernelGGL(k_field_prep, grid, block, 0, stream, rho, node, nx, ny, nz,
                       K / spacing[0], K / spacing[1], K / spacing[2], K);
    return (int)hipGetLastError();
}

int launch_clear_u64(unsigned long long *p, int64_t n, hipStream_t stream)
{
    if (n <= 0) return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_clear_u64, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
    return (int)hipGetLastError();
}

}  // namespace pbr
