// Readout of the Q32.32 sensor accumulator: raw copy, float (value * 2^-32) or 16-bit
// (min(65535, round-half-even(value * gain)), gain = 65535 / largest value unless given), the
// 16-bit dynamic range the paper reaches with about 1e4 rays per source (sec. 3.4).
// Both kernels stream W*H*8 bytes in and 2-8 bytes out per pixel: HBM-bound.
#include "pbr_internal.h"

namespace pbr {
namespace {

__global__ void __launch_bounds__(256)
k_max_u64(const unsigned long long *__restrict__ a, int64_t n, unsigned long long *out)
{
    unsigned long long m = 0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        m = a[q] > m ? a[q] : m;
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_down(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m) atomicMax(out, m);
}

__global__ void __launch_bounds__(256)
k_readout(const unsigned long long *__restrict__ a, int64_t n, int fmt, void *out, double gain,
          const unsigned long long *__restrict__ maxp)
{
    double g = gain;
    if (fmt == PBR_FMT_U16 && !(g > 0.0)) {
        const double mx = (double)(*maxp) * (1.0 / 4294967296.0);
        g = mx > 0.0 ? 65535.0 / mx : 0.0;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const unsigned long long v = a[q];
        if (fmt == PBR_FMT_RAW_U64) {
            ((unsigned long long *)out)[q] = v;
        } else if (fmt == PBR_FMT_F32) {
            ((float *)out)[q] = (float)((double)v * (1.0 / 4294967296.0));
        } else {
            double r = rint((double)v * (1.0 / 4294967296.0) * g);
            r = r < 65535.0 ? r : 65535.0;
            ((unsigned short *)out)[q] = (unsigned short)r;
        }
    }
}

}  // namespace

int launch_readout(const unsigned long long *accum, int64_t npx, int fmt, void *out,
                   double gain, unsigned long long *counters, hipStream_t stream)
{
    int64_t blocks = (npx + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    unsigned long long *maxp = counters + CNT_MAXPIX;
    if (fmt == PBR_FMT_U16 && !(gain > 0.0)) {
        int e = launch_clear_u64(maxp, 1, stream);
        if (e) return e;
        hipLaunchKernelGGL(k_max_u64, dim3((unsigned)blocks), dim3(256), 0, stream, accum, npx, maxp);
        e = (int)hipGetLastError();
        if (e) return e;
    }
    hipLaunchKernelGGL(k_readout, dim3((unsigned)blocks), dim3(256), 0, stream, accum, npx, fmt,
                       out, gain, maxp);
    return (int)hipGetLastError();
}

}  // namespace pbr
