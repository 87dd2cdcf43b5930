// Field preparation (sec. 3.2): Gladstone-Dale n = K rho + 1 (eq. 1) and the refractive-index
// gradient at the grid nodes (central differences inside, second-order one-sided differences on
// the faces), stored per cell as the coefficients of the trilinear interpolant of
// (n - 1, grad n) over the cell's eight corners (layout in pbr_internal.h), or per node.
//
// One thread per cell; all arithmetic in FP64, rounded once to float32 on output.  The kernel
// streams rho (4 B per node, neighbours from cache) and writes 128 B per cell: HBM-bound.
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

// Per-node values (n - 1, dn/dx, dn/dy, dn/dz) for the node layout: one thread per node.
__global__ void __launch_bounds__(256)
k_field_nodes(const float *__restrict__ rho, float4 *__restrict__ nodes, int nx, int ny, int nz, double kx,
              double ky, double kz, double K)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= nx) return;
    const size_t sy = (size_t)nx, sz = (size_t)nx * (size_t)ny;
    const size_t q = (size_t)k * sz + (size_t)j * sy + (size_t)i;
    nodes[q] = make_float4((float)(K * (double)rho[q]), (float)(kx * index_derivative(rho, q, 1, i, nx)),
                           (float)(ky * index_derivative(rho, q, sy, j, ny)),
                           (float)(kz * index_derivative(rho, q, sz, k, nz)));
}

// cells = null: only the per-brick steepness (node layout).
__global__ void __launch_bounds__(256)
k_field_prep(const float *__restrict__ rho, float4 *__restrict__ cells, unsigned *__restrict__ brick_gmax,
             int nx, int ny, int nz, double kx, double ky, double kz, double K)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= nx - 1) return;
    const size_t sx = 1, sy = (size_t)nx, sz = (size_t)nx * (size_t)ny;
    // corner values v[corner][quantity], corner = dx + 2 dy + 4 dz
    double v[8][4];
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
        const int ii = i + (corner & 1), jj = j + ((corner >> 1) & 1), kk = k + (corner >> 2);
        const size_t q = (size_t)kk * sz + (size_t)jj * sy + (size_t)ii;
        v[corner][0] = K * (double)rho[q];
        v[corner][1] = kx * index_derivative(rho, q, sx, ii, nx);
        v[corner][2] = ky * index_derivative(rho, q, sy, jj, ny);
        v[corner][3] = kz * index_derivative(rho, q, sz, kk, nz);
    }
    // steepness of the cell: largest |grad n| at its corners, folded into its brick
    double gm = 0.0;
#pragma unroll
    for (int corner = 0; corner < 8; ++corner)
        gm = fmax(gm, sqrt(v[corner][1] * v[corner][1] + v[corner][2] * v[corner][2] + v[corner][3] * v[corner][3]));
    {
        const int nbx = (nx - 1 + kBrick - 1) / kBrick, nby = (ny - 1 + kBrick - 1) / kBrick;
        const size_t b = ((size_t)(k / kBrick) * nby + (size_t)(j / kBrick)) * nbx + (size_t)(i / kBrick);
        const float gf = (float)gm;
        if (gf > 0.0f) atomicMax(brick_gmax + b, __float_as_uint(gf));  // non-negative floats order as uints
    }
    if (!cells) return;
    double c[8][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const double f000 = v[0][m], f100 = v[1][m], f010 = v[2][m], f110 = v[3][m];
        const double f001 = v[4][m], f101 = v[5][m], f011 = v[6][m], f111 = v[7][m];
        c[0][m] = f000;
        c[1][m] = f100 - f000;
        c[2][m] = f010 - f000;
        c[3][m] = f001 - f000;
        c[4][m] = f110 - f100 - f010 + f000;
        c[5][m] = f101 - f100 - f001 + f000;
        c[6][m] = f011 - f010 - f001 + f000;
        c[7][m] = f111 - f110 - f101 - f011 + f100 + f010 + f001 - f000;
    }
    const size_t cell = ((size_t)k * (size_t)(ny - 1) + (size_t)j) * (size_t)(nx - 1) + (size_t)i;
    float4 *out = cells + cell * kCellFloat4;
#pragma unroll
    for (int m = 0; m < 8; ++m)
        out[m] = make_float4((float)c[m][0], (float)c[m][1], (float)c[m][2], (float)c[m][3]);
}

// Fingerprint of a field: sum over its 32-bit words w_k of SplitMix64's finaliser applied to
// (k << 32 | w_k), wrapping mod 2^64 (integer atomics: independent of the order of the blocks).
__global__ void __launch_bounds__(256) k_checksum(const unsigned *__restrict__ w, int64_t n,
                                                  unsigned long long *__restrict__ out)
{
    unsigned long long acc = 0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        unsigned long long z = ((unsigned long long)k << 32) ^ (unsigned long long)w[k];
        z += 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        acc += z ^ (z >> 31);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63u) == 0)
        __hip_atomic_fetch_add(out, acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sets *bad when any density value is not finite.
__global__ void __launch_bounds__(256) k_check_finite(const float *__restrict__ rho, int64_t n,
                                                      unsigned long long *__restrict__ bad)
{
    bool ok = true;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) ok = ok && isfinite(rho[k]);
    if (__ballot(!ok) != 0ull && (threadIdx.x & 63u) == 0)
        __hip_atomic_fetch_add(bad, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256) k_clear_u64(unsigned long long *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = 0ull;
}

}  // namespace

int launch_field_prep(const float *rho, float4 *cells, unsigned *brick_gmax, int nx, int ny, int nz,
                      const double spacing[3], double K, hipStream_t stream, bool nodes)
{
    dim3 block(256);
    dim3 grid((unsigned)((nx - 1 + 255) / 256), (unsigned)(ny - 1), (unsigned)(nz - 1));
    hipLaunchKernelGGL(k_field_prep, grid, block, 0, stream, rho, nodes ? nullptr : cells, brick_gmax, nx, ny, nz,
                       K / spacing[0], K / spacing[1], K / spacing[2], K);
    if (nodes) {
        dim3 ngrid((unsigned)((nx + 255) / 256), (unsigned)ny, (unsigned)nz);
        hipLaunchKernelGGL(k_field_nodes, ngrid, block, 0, stream, rho, cells, nx, ny, nz, K / spacing[0],
                           K / spacing[1], K / spacing[2], K);
    }
    return (int)hipGetLastError();
}

int launch_field_checksum(const void *field, size_t bytes, unsigned long long *out, hipStream_t stream)
{
    const int64_t n = (int64_t)(bytes / 4);
    int e = launch_clear_u64(out, 1, stream);
    if (e || n == 0) return e;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_checksum, dim3((unsigned)blocks), dim3(256), 0, stream, (const unsigned *)field, n, out);
    return (int)hipGetLastError();
}

int launch_check_finite(const float *rho, int64_t n, unsigned long long *bad, hipStream_t stream)
{
    int e = launch_clear_u64(bad, 1, stream);
    if (e || n <= 0) return e;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, stream, rho, n, bad);
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
