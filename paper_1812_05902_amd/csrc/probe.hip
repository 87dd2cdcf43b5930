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

// ------------------------------------------------------------------ peaks of the roofline
// Measured ceilings for the rooflines the benchmark reports: the vector FMA issue rate (FP32 with
// packed FP32 instructions disabled, as the library is built, and FP64), read bandwidth from a
// buffer that fits the L2 caches or one that does not (HBM), coalesced or one 16-byte load per
// lane at scattered lines (the shape of a field gather), and LDS read bandwidth.

namespace {

constexpr int kFmaChains = 8;

template <typename T>
__global__ void __launch_bounds__(256) k_probe_fma(T *__restrict__ out, int iters, T a, T b)
{
    T x[kFmaChains];
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) x[k] = (T)(threadIdx.x + k) * (T)1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < kFmaChains; ++k) x[k] = fma(x[k], a, b);
    }
    T s = (T)0;
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) s += x[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Reads total4 float4 from buf (n4 = power of two float4); coalesced: consecutive lanes read
// consecutive float4; scattered: every lane reads one float4 of its own 128-byte line.
template <bool SCATTER>
__global__ void __launch_bounds__(256) k_probe_read(const float4 *__restrict__ buf, int64_t mask4, int64_t per_thread,
                                                    float *__restrict__ out)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    float ax = 0.0f, ay = 0.0f, az = 0.0f, aw = 0.0f;
    int64_t i = tid;
    for (int64_t k = 0; k < per_thread; k += 4) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int64_t j = i + (int64_t)u * nth;
            if (SCATTER) j = (j * 8 + (j >> 6) * 3) & mask4;  // one float4 per 128-byte line, lanes 128 B apart
            else j &= mask4;
            v[u] = buf[j];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) { ax += v[u].x; ay += v[u].y; az += v[u].z; aw += v[u].w; }
        i += 4 * nth;
    }
    out[tid] = ax + ay + az + aw;
}

__global__ void __launch_bounds__(256) k_probe_lds(float *__restrict__ out, int iters)
{
    __shared__ float4 s[2048];  // 32 KiB
    for (int k = threadIdx.x; k < 2048; k += blockDim.x) s[k] = make_float4((float)k, 0.0f, 0.0f, 0.0f);
    __syncthreads();
    float ax = 0.0f, ay = 0.0f, az = 0.0f, aw = 0.0f;
    int idx = threadIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 v = s[(idx + u * 256) & 2047];
            ax += v.x; ay += v.y; az += v.z; aw += v.w;
        }
        idx = (idx + 64) & 2047;
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = ax + ay + az + aw;
}

// Times launch() once after a warm-up launch on the null stream; ms out.
template <typename L>
int time_launch(L launch, float *ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PBR_ERR_HIP;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        launch();
        (void)hipEventRecord(e0, nullptr);
        launch();
        (void)hipEventRecord(e1, nullptr);
        if (hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(ms, e0, e1) == hipSuccess && *ms > 0.0f)
            rc = PBR_OK;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

struct ProbeDevice {
    int prev = -1, ncu = 256;
    bool ok = false;
    explicit ProbeDevice(int device)
    {
        if (hipGetDevice(&prev) != hipSuccess) { prev = -1; return; }
        if (hipSetDevice(device) != hipSuccess) return;
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
        ok = true;
    }
    ~ProbeDevice()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" int pbr_probe_fma_rate(int device, int fp64, double *flop_per_s)
{
    if (!flop_per_s) return PBR_ERR_ARG;
    ProbeDevice pd(device);
    if (!pd.ok) return PBR_ERR_ARG;
    const unsigned blocks = (unsigned)pd.ncu * 16u;  // four 256-thread blocks per SIMD
    const int iters = fp64 ? 2048 : 4096;
    void *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * 8) != hipSuccess) return PBR_ERR_HIP;
    float ms = 0.0f;
    int rc;
    if (fp64)
        rc = time_launch([&] { hipLaunchKernelGGL(k_probe_fma<double>, dim3(blocks), dim3(256), 0, nullptr,
                                                  (double *)out, iters, 0.999999, 1e-7); }, &ms);
    else
        rc = time_launch([&] { hipLaunchKernelGGL(k_probe_fma<float>, dim3(blocks), dim3(256), 0, nullptr,
                                                  (float *)out, iters, 0.999999f, 1e-7f); }, &ms);
    (void)hipFree(out);
    if (rc) return rc;
    const double flop = 2.0 * (double)blocks * 256.0 * (double)iters * 8.0 * (double)kFmaChains;
    *flop_per_s = flop / ((double)ms * 1e-3);
    return PBR_OK;
}

extern "C" int pbr_probe_read_bandwidth(int device, int64_t buffer_bytes, int64_t total_bytes, int scattered,
                                        double *bytes_per_s)
{
    if (!bytes_per_s || buffer_bytes < 65536 || (buffer_bytes & (buffer_bytes - 1)) || total_bytes < buffer_bytes)
        return PBR_ERR_ARG;
    ProbeDevice pd(device);
    if (!pd.ok) return PBR_ERR_ARG;
    const unsigned blocks = (unsigned)pd.ncu * 16u;
    const int64_t nth = (int64_t)blocks * 256;
    int64_t per_thread = (total_bytes / 16 + nth - 1) / nth;
    per_thread = (per_thread + 3) / 4 * 4;
    void *buf = nullptr, *out = nullptr;
    int rc = PBR_ERR_HIP;
    if (hipMalloc(&buf, (size_t)buffer_bytes) == hipSuccess && hipMalloc(&out, (size_t)nth * 4) == hipSuccess &&
        hipMemset(buf, 0, (size_t)buffer_bytes) == hipSuccess) {
        const int64_t mask4 = buffer_bytes / 16 - 1;
        float ms = 0.0f;
        if (scattered)
            rc = time_launch([&] { hipLaunchKernelGGL(k_probe_read<true>, dim3(blocks), dim3(256), 0, nullptr,
                                                      (const float4 *)buf, mask4, per_thread, (float *)out); }, &ms);
        else
            rc = time_launch([&] { hipLaunchKernelGGL(k_probe_read<false>, dim3(blocks), dim3(256), 0, nullptr,
                                                      (const float4 *)buf, mask4, per_thread, (float *)out); }, &ms);
        if (!rc) *bytes_per_s = (double)nth * (double)per_thread * 16.0 / ((double)ms * 1e-3);
    }
    if (buf) (void)hipFree(buf);
    if (out) (void)hipFree(out);
    return rc;
}

extern "C" int pbr_probe_lds_bandwidth(int device, double *bytes_per_s)
{
    if (!bytes_per_s) return PBR_ERR_ARG;
    ProbeDevice pd(device);
    if (!pd.ok) return PBR_ERR_ARG;
    const unsigned blocks = (unsigned)pd.ncu * 16u;
    const int iters = 4096;
    void *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * 4) != hipSuccess) return PBR_ERR_HIP;
    float ms = 0.0f;
    const int rc = time_launch([&] { hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(256), 0, nullptr,
                                                        (float *)out, iters); }, &ms);
    (void)hipFree(out);
    if (rc) return rc;
    *bytes_per_s = (double)blocks * 256.0 * (double)iters * 8.0 * 16.0 / ((double)ms * 1e-3);
    return PBR_OK;
}
