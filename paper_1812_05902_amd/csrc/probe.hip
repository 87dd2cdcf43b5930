// Calibration probe: the rate of 64-bit integer atomic additions to device memory that the sensor
// deposit relies on (sec. 3.4 sums spot contributions; here they are Q32.32 integers added with
// atomics).  Used to state the deposit kernel's atomic throughput against what the chip sustains.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbr.h"

namespace {

__global__ void __launch_bounds__(256) k_probe_atomics(unsigned long long *__restrict__ buf, int64_t n_slots,
                                                       int64_t n_updates)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_updates; i += stride) {
        // neighbouring threads hit neighbouring slots (as a spot's pixels do), blocks spread out
        uint64_t h = (uint64_t)(i >> 8) * 0x9E3779B97F4A7C15ull;
        h ^= h >> 29;
        const int64_t slot = (int64_t)((h + (uint64_t)(i & 255)) % (uint64_t)n_slots);
        atomicAdd(buf + slot, 1ull);
    }
}

}  // namespace

extern "C" int pbr_probe_u64_atomics(int device, int64_t n_slots, int64_t n_updates, double *updates_per_s)
{
    if (n_slots < 1 || n_updates < 1 || !updates_per_s) return PBR_ERR_ARG;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return PBR_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return PBR_ERR_ARG;
    unsigned long long *buf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PBR_ERR_HIP;
    if (hipMalloc(&buf, (size_t)n_slots * 8) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess && hipMemset(buf, 0, (size_t)n_slots * 8) == hipSuccess) {
        int ncu = 256;
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
        const dim3 grid((unsigned)ncu * 8u), block(256);
        hipLaunchKernelGGL(k_probe_atomics, grid, block, 0, nullptr, buf, n_slots, n_updates);  // warm-up
        (void)hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(k_probe_atomics, grid, block, 0, nullptr, buf, n_slots, n_updates);
        (void)hipEventRecord(e1, nullptr);
        float ms = 0.0f;
        if (hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f) {
            *updates_per_s = (double)n_updates / ((double)ms * 1e-3);
            rc = PBR_OK;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
    (void)hipSetDevice(prev);
    return rc;
}
