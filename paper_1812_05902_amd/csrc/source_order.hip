// Locality order of the sources: the permutation that sorts their positions by Morton code.
// The trace takes its sources in this order (sec. 3.5: rays of neighbouring sources cross the
// same cells, so tracing them together raises the cache reuse of the field gathers).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "pbr_internal.h"

namespace pbr {
namespace {

// Spreads the low 21 bits of v to every third bit (bit k goes to bit 3k).
__device__ __forceinline__ unsigned long long spread3(unsigned long long v)
{
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Key of source q: its position in the box [lo, lo + ext] on a 2^21 grid per axis (clamped onto
// the box), bits interleaved x, y, z from the lowest; value: q.
__global__ void __launch_bounds__(256) k_morton_keys(const float4 *__restrict__ src, int n, double lo0, double lo1,
                                                     double lo2, double ie0, double ie1, double ie2,
                                                     unsigned long long *__restrict__ keys, int64_t *__restrict__ idx)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float4 s = src[q];
    const double p[3] = {((double)s.x - lo0) * ie0, ((double)s.y - lo1) * ie1, ((double)s.z - lo2) * ie2};
    unsigned long long key = 0ull;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double t = p[a] * 2097152.0;
        t = t > 0.0 ? (t < 2097151.0 ? t : 2097151.0) : 0.0;  // NaN goes to 0 as well
        key |= spread3((unsigned long long)t) << a;
    }
    keys[q] = key;
    idx[q] = q;
}

struct OrderScratch {
    size_t keys_in, keys_out, idx, temp, temp_bytes, total;
};

OrderScratch order_scratch(int n)
{
    OrderScratch o{};
    size_t temp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const unsigned long long *)nullptr,
                                             (unsigned long long *)nullptr, (const int64_t *)nullptr,
                                             (int64_t *)nullptr, n, 0, 63);
    o.keys_in = 0;
    o.keys_out = align256(o.keys_in + (size_t)n * 8);
    o.idx = align256(o.keys_out + (size_t)n * 8);
    o.temp = align256(o.idx + (size_t)n * 8);
    o.temp_bytes = temp;
    o.total = align256(o.temp + temp);
    return o;
}

}  // namespace

size_t morton_order_scratch_bytes(int64_t n)
{
    if (n < 0 || n > 2147483647) return 0;
    return order_scratch((int)(n > 0 ? n : 1)).total;
}

int launch_morton_order(const float4 *src, int64_t n, const double lo[3], const double ext[3], int64_t *order,
                        void *ws, hipStream_t stream)
{
    if (n <= 0) return 0;
    const OrderScratch o = order_scratch((int)n);
    unsigned char *w = (unsigned char *)ws;
    unsigned long long *keys_in = (unsigned long long *)(w + o.keys_in);
    unsigned long long *keys_out = (unsigned long long *)(w + o.keys_out);
    int64_t *idx = (int64_t *)(w + o.idx);
    double ie[3];
    for (int a = 0; a < 3; ++a) ie[a] = ext[a] > 0.0 ? 1.0 / ext[a] : 0.0;
    hipLaunchKernelGGL(k_morton_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src, (int)n, lo[0],
                       lo[1], lo[2], ie[0], ie[1], ie[2], keys_in, idx);
    int e = (int)hipGetLastError();
    if (e) return e;
    size_t temp = o.temp_bytes;
    return (int)hipcub::DeviceRadixSort::SortPairs(w + o.temp, temp, keys_in, keys_out, idx, order, (int)n, 0, 63,
                                                   stream);
}

}  // namespace pbr
