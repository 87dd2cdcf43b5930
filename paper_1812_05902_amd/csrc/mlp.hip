// Kernels of the ray-surrogate network 6 -> 256 -> 256 -> 256 -> 256 -> 6 (GELU, tanh form):
// the input layer in FP32 (entry positions need more than bfloat16's 8 bits), the three hidden
// 256 x 256 layers and the output layer as bfloat16 matrix products on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), the backward pass (error propagation, weight
// and bias gradients) and Adam on FP32 master weights with bfloat16 shadow copies.
#include "mlp_internal.h"

namespace pbr {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2 / pi)
constexpr float kGeluA = 0.044715f;

// GELU, tanh form, through the identity (1 + tanh u) / 2 = 1 / (1 + exp(-2 u)) with
// -2 u = z (k1 + k3 z^2) log2(e)-scaled, so that one hardware 2^x and one reciprocal (about 1 ulp
// each) and three multiply(-add)s replace a branchy tanh.  Saturates correctly: 2^x overflow gives
// 0, underflow gives z.
constexpr float kGeluK1 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;             // -2 c log2 e
constexpr float kGeluK3 = -2.0f * 0.7978845608028654f * 0.044715f * 1.4426950408889634f;  // -2 c a log2 e
__device__ __forceinline__ float gelu_sig(float z)
{
    const float e = __builtin_amdgcn_exp2f(z * __builtin_fmaf(z * z, kGeluK3, kGeluK1));
    return __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ float gelu(float z) { return z * gelu_sig(z); }

// d/dz of z s(z), s = (1 + tanh u) / 2: s + 2 z s (1 - s) u'(z), u' = c (1 + 3 a z^2)
__device__ __forceinline__ float gelu_grad(float z)
{
    const float sg = gelu_sig(z);
    return sg + 2.0f * z * sg * (1.0f - sg) * kGeluC * (1.0f + 3.0f * kGeluA * z * z);
}

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// C[m][n] = sum_k A[m][k] W[n][k] (+ bias[n]); A: M x K, W: N x K, both bf16, k contiguous.
// Block 256 threads = 4 waves in 2 x 2, block tile 64 x 64, wave tile 32 x 32 = 2 x 2 matrix-core
// tiles of 16 x 16.  Operand layout of the 16x16x32 instruction: lane l supplies row (A) or
// column (B) l % 16 and the 8 consecutive k starting at 8 (l / 16); the 4 results of lane l are
// rows 4 (l / 16) + t, column l % 16.  M, N multiples of 64, K a multiple of 32.
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(const unsigned short *__restrict__ A, int lda,
                                                 const unsigned short *__restrict__ W, int ldw,
                                                 const float *__restrict__ bias, int K, float *__restrict__ Cf,
                                                 int ldc, unsigned short *__restrict__ Cb, int ldcb,
                                                 const float *__restrict__ Zin, int n_valid,
                                                 const unsigned long long *__restrict__ live)
{
    // rows beyond the live count (read on the device) are skipped whole blocks at a time
    if (live && (unsigned long long)blockIdx.y * 64ull >= *live) return;
    // split K (plain products only): block z takes k in [z K, (z + 1) K) and writes slice z of Cf
    A += (size_t)blockIdx.z * K;
    W += (size_t)blockIdx.z * K;
    if (Cf) Cf += (size_t)blockIdx.z * gridDim.y * 64 * ldc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int r = lane & 15, kg = lane >> 4;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const unsigned short *a0 = A + (size_t)(m0 + r) * lda + 8 * kg;
    const unsigned short *a1 = A + (size_t)(m0 + 16 + r) * lda + 8 * kg;
    const unsigned short *w0 = W + (size_t)(n0 + r) * ldw + 8 * kg;
    const unsigned short *w1 = W + (size_t)(n0 + 16 + r) * ldw + 8 * kg;
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 fa0 = *(const bf16x8 *)(a0 + k0);
        const bf16x8 fa1 = *(const bf16x8 *)(a1 + k0);
        const bf16x8 fw0 = *(const bf16x8 *)(w0 + k0);
        const bf16x8 fw1 = *(const bf16x8 *)(w1 + k0);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fw0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fw1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fw0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fw1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + 16 * j + r;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int m = m0 + 16 * i + 4 * kg + t;
                float z = acc[i][j][t];
                if (EPI == EPI_BIAS_GELU || EPI == EPI_BIAS_Z_GELU) z += bias[n];
                if (EPI == EPI_BIAS_OUT) z += n < n_valid ? bias[n] : 0.0f;
                if (EPI == EPI_BIAS_GELU) {
                    Cb[(size_t)m * ldcb + n] = bf16_bits(gelu(z));
                } else if (EPI == EPI_BIAS_Z_GELU) {
                    Cf[(size_t)m * ldc + n] = z;
                    Cb[(size_t)m * ldcb + n] = bf16_bits(gelu(z));
                } else if (EPI == EPI_BIAS_OUT) {
                    if (n < n_valid) Cf[(size_t)m * ldc + n] = z;
                } else if (EPI == EPI_GELU_BACK) {
                    // z is dL/da of the layer below; dL/dz = dL/da * g'(z_below)
                    const float dz = z * gelu_grad(Zin[(size_t)m * ldc + n]);
                    Cf[(size_t)m * ldc + n] = dz;
                    Cb[(size_t)m * ldcb + n] = bf16_bits(dz);
                } else {  // EPI_PLAIN
                    Cf[(size_t)m * ldc + n] = z;
                }
            }
        }
}

// Input layer in FP32: z1 = x W1^T + b1, a1 = bf16(g(z1)).  One thread per (row, unit).
__global__ void __launch_bounds__(256) k_layer1(const float *__restrict__ x, const float *__restrict__ W1,
                                                const float *__restrict__ b1, int64_t rows,
                                                float *__restrict__ z1, unsigned short *__restrict__ a1,
                                                const unsigned long long *__restrict__ live)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * kHidden) return;
    // whole 64-row groups past the live count are skipped, as in the matrix products
    if (live && (unsigned long long)(q / (kHidden * 64)) * 64ull >= *live) return;
    const int64_t m = q / kHidden;
    const int n = (int)(q % kHidden);
    float z = b1[n];
#pragma unroll
    for (int k = 0; k < kIn; ++k) z += x[m * kIn + k] * W1[n * kIn + k];
    if (z1) z1[q] = z;
    a1[q] = bf16_bits(gelu(z));
}

// Output errors of the mean squared error: dy = 2 (y - t) / (rows * 6); per-block loss sums.
__global__ void __launch_bounds__(256) k_out_error(const float *__restrict__ y, const float *__restrict__ t,
                                                   int64_t rows, float *__restrict__ dy, float *__restrict__ loss_part)
{
    __shared__ float s[256];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (q < rows * kOut) {
        const float d = y[q] - t[q];
        dy[q] = 2.0f * d / (float)(rows * kOut);
        l = d * d;
    }
    s[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = s[0];
}

// dL/da4 = dy W5 (K = 6, FP32 master weights), then dL/dz4 = dL/da4 g'(z4) in f32 and bf16.
__global__ void __launch_bounds__(256) k_out_back(const float *__restrict__ dy, const float *__restrict__ W5,
                                                  const float *__restrict__ z4, int64_t rows,
                                                  float *__restrict__ dz, unsigned short *__restrict__ dzb)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * kHidden) return;
    const int64_t m = q / kHidden;
    const int n = (int)(q % kHidden);
    float da = 0.0f;
#pragma unroll
    for (int o = 0; o < kOut; ++o) da += dy[m * kOut + o] * W5[o * kHidden + n];
    const float d = da * gelu_grad(z4[q]);
    dz[q] = d;
    dzb[q] = bf16_bits(d);
}

// out[c][r] = in[r][c] for a rows x cols bf16 matrix (32 x 32 tiles through LDS).
__global__ void __launch_bounds__(256) k_transpose(const unsigned short *__restrict__ in, int64_t rows, int cols,
                                                   unsigned short *__restrict__ out)
{
    __shared__ unsigned short tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32;
    const int c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k;
        const int c = c0 + tx;
        tile[k][tx] = (r < rows && c < cols) ? in[r * cols + c] : (unsigned short)0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int c = c0 + k;
        const int64_t r = r0 + tx;
        if (c < cols && r < rows) out[(int64_t)c * rows + r] = tile[tx][k];
    }
}

// Reductions over the rows of a batch against one 256-wide operand (weight gradients of the
// 6-wide layers and bias gradients), in two passes with a fixed summation order.  Pass 1: block y
// takes rows [y RB, (y + 1) RB); thread w owns column w of the wide operand (row reads are
// coalesced) and accumulates, per small column s, wide[m][w] * small[m][s] (ns of them), the
// plain column sum of wide[.][w] (if ones), and, in thread 0, the column sums of small (if
// small_sums).  Pass 2 adds the blocks in order and scatters: products to G ([s][w] if
// small_major, else [w][s]), wide sums to gw, small sums to gs.
template <bool WIDE_BF16>
__global__ void __launch_bounds__(256) k_wide_part(const void *__restrict__ wide, int64_t rows,
                                                   const float *__restrict__ small, int ns, int ones,
                                                   int small_sums, int64_t rb, float *__restrict__ part)
{
    const int w = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * rb;
    const int64_t m1 = m0 + rb < rows ? m0 + rb : rows;
    float acc[kOut + 1], accs[kOut];
#pragma unroll
    for (int q = 0; q <= kOut; ++q) acc[q] = 0.0f;
#pragma unroll
    for (int q = 0; q < kOut; ++q) accs[q] = 0.0f;
#pragma unroll 8
    for (int64_t m = m0; m < m1; ++m) {
        float v;
        if (WIDE_BF16) v = __uint_as_float(((unsigned)((const unsigned short *)wide)[m * kHidden + w]) << 16);
        else v = ((const float *)wide)[m * kHidden + w];
#pragma unroll
        for (int q = 0; q < kOut; ++q)
            if (q < ns) {
                const float sv = small[m * ns + q];
                acc[q] += v * sv;
                accs[q] += sv;
            }
        acc[kOut] += v;
    }
    const int stride = kHidden * (ns + ones) + (small_sums ? ns : 0);
    float *o = part + (size_t)blockIdx.x * stride;
    for (int q = 0; q < ns; ++q) o[w * (ns + ones) + q] = acc[q];
    if (ones) o[w * (ns + ones) + ns] = acc[kOut];
    if (small_sums && w == 0)
        for (int q = 0; q < ns; ++q) o[kHidden * (ns + ones) + q] = accs[q];
}

// Block: 32 outputs x 8 lanes; lane g sums blocks g, g + 8, ... (loads in flight), then the 8
// lane sums are added in a fixed tree.
__global__ void __launch_bounds__(256) k_wide_final(const float *__restrict__ part, int nblocks, int ns, int ones,
                                                    int small_sums, int small_major, float *__restrict__ G,
                                                    float *__restrict__ gw, float *__restrict__ gs)
{
    __shared__ float red[8][32];
    const int stride = kHidden * (ns + ones) + (small_sums ? ns : 0);
    const int ql = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int q = blockIdx.x * 32 + ql;
    float a = 0.0f;
    if (q < stride) {
#pragma unroll 8
        for (int y = g; y < nblocks; y += 8) a += part[(size_t)y * stride + q];
    }
    red[g][ql] = a;
    __syncthreads();
    if (g == 0 && q < stride) {
        const float t = ((red[0][ql] + red[1][ql]) + (red[2][ql] + red[3][ql])) +
                        ((red[4][ql] + red[5][ql]) + (red[6][ql] + red[7][ql]));
        if (q < kHidden * (ns + ones)) {
            const int w = q / (ns + ones), k = q % (ns + ones);
            if (k < ns) G[small_major ? k * kHidden + w : w * ns + k] = t;
            else gw[w] = t;
        } else {
            gs[q - kHidden * (ns + ones)] = t;
        }
    }
}

// C = sum of the nsplit slices of part (each n floats), in slice order.
__global__ void __launch_bounds__(256) k_split_sum(const float *__restrict__ part, int nsplit, int64_t n,
                                                   float *__restrict__ C)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    float a = 0.0f;
#pragma unroll 16
    for (int z = 0; z < nsplit; ++z) a += part[(size_t)z * n + q];
    C[q] = a;
}

// Adam on the flat FP32 parameters (Kingma & Ba), then the bf16 copies the products read:
// W2..W4 (and their transposes) and W5 padded to 64 rows.
__global__ void __launch_bounds__(256) k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int64_t n, float lr,
                                              float beta1, float beta2, float eps, float c1, float c2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = beta1 * m[q] + (1.0f - beta1) * gq;
    const float vq = beta2 * v[q] + (1.0f - beta2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// Adam with the step number read on the device (graph replays): t = *step + 1, learning rate on a
// cosine from lr_max (first step) to lr_min (step total - 1).
__global__ void __launch_bounds__(256) k_adam_sched(float *__restrict__ p, const float *__restrict__ g,
                                                    float *__restrict__ m, float *__restrict__ v, int64_t n,
                                                    const int *__restrict__ step, int total, float lr_max,
                                                    float lr_min, float beta1, float beta2, float eps)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int k = *step;
    const float ph = total > 1 ? (float)k / (float)(total - 1) : 0.0f;
    const float lr = lr_min + 0.5f * (lr_max - lr_min) * (1.0f + cosf(3.14159265358979f * ph));
    const float c1 = 1.0f - powf(beta1, (float)(k + 1)), c2 = 1.0f - powf(beta2, (float)(k + 1));
    const float gq = g[q];
    const float mq = beta1 * m[q] + (1.0f - beta1) * gq;
    const float vq = beta2 * v[q] + (1.0f - beta2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

__global__ void k_step_advance(int *step)
{
    if (threadIdx.x == 0) *step += 1;
}

__global__ void __launch_bounds__(256) k_shadow(const float *__restrict__ p, unsigned short *__restrict__ w2,
                                                unsigned short *__restrict__ w2t, unsigned short *__restrict__ w3,
                                                unsigned short *__restrict__ w3t, unsigned short *__restrict__ w4,
                                                unsigned short *__restrict__ w4t, unsigned short *__restrict__ w5)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < kHidden * kHidden) {
        const int o = q / kHidden, i = q % kHidden;
        const unsigned short b2 = bf16_bits(p[kOffW2 + q]), b3 = bf16_bits(p[kOffW3 + q]), b4 = bf16_bits(p[kOffW4 + q]);
        w2[q] = b2; w3[q] = b3; w4[q] = b4;
        w2t[i * kHidden + o] = b2; w3t[i * kHidden + o] = b3; w4t[i * kHidden + o] = b4;
    }
    if (q < kOutPad * kHidden) {
        const int o = q / kHidden;
        w5[q] = o < kOut ? bf16_bits(p[kOffW5 + q]) : (unsigned short)0;
    }
}

// Mean of the squared errors of one batch from the per-block sums of k_out_error, into out[0]
// (or out[*step] when step is given).
__global__ void __launch_bounds__(256) k_loss_mean(const float *__restrict__ part, int nparts, float inv_count,
                                                   float *__restrict__ out, const int *__restrict__ step)
{
    if (step) out += *step;
    __shared__ float s[256];
    float a = 0.0f;
    for (int i = threadIdx.x; i < nparts; i += 256) a += part[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0] * inv_count;
}

// Whole forward pass in one launch for inference.  A block of eight waves takes 128 rows
// (samples) and keeps their activations in LDS as bf16 [sample][unit] (rows padded to 264
// elements so that the 16 samples one matrix-core operand read touches fall in distinct banks).
// Products are computed transposed, Z^T = W A^T: the weights are the A operand (16 B per lane
// from L2, two k steps ahead), the activations the B operand (16 B per lane from LDS), and a
// lane's four results are four consecutive units of one sample, so that bias, GELU and the bf16
// rounding (hardware round-to-nearest-even, two values per instruction) end in one 8-byte LDS
// store per four values.  Wave w owns units 32 w .. 32 w + 31 of all 128 samples (2 x 8 tiles of
// 16 x 16): 64 accumulator registers, so that four waves share each SIMD and one wave's vector
// work (bias, GELU, rounding) overlaps another's matrix-core work.  Layer 1 (K = 6, padded to 8)
// runs in FP32 on the matrix cores (v_mfma_f32_16x16x4_f32, same tiles and result layout).  The
// output layer is 16 (6 used) x 128, each wave taking 16 samples.
constexpr int kFuseRows = 128, kActStride = kHidden + 8, kFuseWaves = 8;

__device__ __forceinline__ unsigned pack_bf16x2(float a, float b)
{
    const bf16x2 p = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(unsigned, p);
}

__global__ void __launch_bounds__(64 * kFuseWaves, 2) k_mlp_infer(const float *__restrict__ x, int64_t rows,
                                                                  const unsigned long long *__restrict__ live,
                                                                  const float *__restrict__ params,
                                                                  const unsigned short *__restrict__ w2,
                                                                  const unsigned short *__restrict__ w3,
                                                                  const unsigned short *__restrict__ w4,
                                                                  const unsigned short *__restrict__ w5,
                                                                  float *__restrict__ y)
{
    __shared__ __attribute__((aligned(16))) unsigned short act[kFuseRows * kActStride];
    __shared__ float xs[kFuseRows * kIn];
    const int64_t row0 = (int64_t)blockIdx.x * kFuseRows;
    int64_t nrow = rows;
    if (live) nrow = (int64_t)(*live < (unsigned long long)rows ? *live : (unsigned long long)rows);
    if (row0 >= nrow) return;
    const int64_t nblk = nrow - row0 < kFuseRows ? nrow - row0 : kFuseRows;
    for (int q = threadIdx.x; q < kFuseRows * kIn; q += 64 * kFuseWaves)
        xs[q] = q < nblk * kIn ? x[row0 * kIn + q] : 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kg = lane >> 4;
    // lane: units 32 w + 16 j + 4 kg + t (t = 0..3) of sample 16 i + r
    auto store_act = [&](floatx4 (&acc)[2][8]) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                uint2 v;
                v.x = pack_bf16x2(gelu(acc[j][i][0]), gelu(acc[j][i][1]));
                v.y = pack_bf16x2(gelu(acc[j][i][2]), gelu(acc[j][i][3]));
                *(uint2 *)(act + (16 * i + r) * kActStride + wave * 32 + 16 * j + 4 * kg) = v;
            }
    };
    {   // layer 1 in FP32 on the matrix cores (v_mfma_f32_16x16x4_f32, K = 6 padded to 8): lane l
        // supplies W1[unit][k] and x[sample][k] for k = kk + l / 16
        floatx4 acc[2][8];
        const float *bias = params + kOffB1 + wave * 32 + 4 * kg;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const float4 b4 = *(const float4 *)(bias + 16 * j);
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[j][i] = floatx4{b4.x, b4.y, b4.z, b4.w};
        }
#pragma unroll
        for (int kk = 0; kk < 8; kk += 4) {
            const int k = kk + kg;
            float wa[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) wa[j] = k < kIn ? params[kOffW1 + (wave * 32 + 16 * j + r) * kIn + k] : 0.0f;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float xb = k < kIn ? xs[(16 * i + r) * kIn + k] : 0.0f;
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[j], xb, acc[j][i], 0, 0, 0);
            }
        }
        store_act(acc);
    }
    __syncthreads();
    for (int l = 0; l < 3; ++l) {
        const unsigned short *W = (l == 0 ? w2 : (l == 1 ? w3 : w4)) + (size_t)(wave * 32 + r) * kHidden + 8 * kg;
        const float *bias = params + (l == 0 ? kOffB2 : (l == 1 ? kOffB3 : kOffB4)) + wave * 32 + 4 * kg;
        // accumulators start at the bias of their unit
        floatx4 acc[2][8];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const float4 b4 = *(const float4 *)(bias + 16 * j);
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[j][i] = floatx4{b4.x, b4.y, b4.z, b4.w};
        }
        // weight fragments two k steps ahead
        bf16x8 fw[2], fn[2], fn2[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            fw[j] = *(const bf16x8 *)(W + j * 16 * kHidden);
            fn[j] = *(const bf16x8 *)(W + j * 16 * kHidden + 32);
        }
#pragma unroll
        for (int k0 = 0; k0 < kHidden; k0 += 32) {
            if (k0 + 64 < kHidden) {
#pragma unroll
                for (int j = 0; j < 2; ++j) fn2[j] = *(const bf16x8 *)(W + j * 16 * kHidden + k0 + 64);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const bf16x8 fa = *(const bf16x8 *)(act + (16 * i + r) * kActStride + 8 * kg + k0);
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[j], fa, acc[j][i], 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                fw[j] = fn[j];
                fn[j] = fn2[j];
            }
        }
        __syncthreads();  // every wave has read this layer's inputs
        store_act(acc);
        __syncthreads();
    }
    {   // output layer: 16 (padded) outputs of samples 16 w .. 16 w + 15
        floatx4 acc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        const unsigned short *W = w5 + (size_t)r * kHidden + 8 * kg;
        for (int k0 = 0; k0 < kHidden; k0 += 32) {
            const bf16x8 fw = *(const bf16x8 *)(W + k0);
            const bf16x8 fa = *(const bf16x8 *)(act + (16 * wave + r) * kActStride + 8 * kg + k0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw, fa, acc, 0, 0, 0);
        }
        // lane: outputs 4 kg + t of sample 16 w + r
        const int m = 16 * wave + r;
        if (kg < 2 && m < nblk) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int o = 4 * kg + t;
                if (o < kOut) y[(row0 + m) * kOut + o] = acc[t] + params[kOffB5 + o];
            }
        }
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Rows per block of the wide reductions and the resulting block count (at most kWideBlocks).
constexpr int kWideBlocks = 256;
inline int64_t wide_rows_per_block(int64_t rows) { return (rows + kWideBlocks - 1) / kWideBlocks; }

int wide_reduce(const void *wide, bool wide_bf16, int64_t rows, const float *small, int ns, bool ones,
                bool small_sums, bool small_major, float *G, float *gw, float *gs, float *part, hipStream_t s)
{
    const int64_t rb = wide_rows_per_block(rows);
    const int nb = (int)((rows + rb - 1) / rb);
    if (wide_bf16)
        hipLaunchKernelGGL(k_wide_part<true>, dim3((unsigned)nb), dim3(256), 0, s, wide, rows, small, ns, (int)ones,
                           (int)small_sums, rb, part);
    else
        hipLaunchKernelGGL(k_wide_part<false>, dim3((unsigned)nb), dim3(256), 0, s, wide, rows, small, ns, (int)ones,
                           (int)small_sums, rb, part);
    const int stride = kHidden * (ns + (ones ? 1 : 0)) + (small_sums ? ns : 0);
    hipLaunchKernelGGL(k_wide_final, dim3((unsigned)((stride + 31) / 32)), dim3(256), 0, s, (const float *)part, nb, ns,
                       (int)ones, (int)small_sums, (int)small_major, G, gw, gs);
    return (int)hipGetLastError();
}

template <int EPI>
int gemm(const unsigned short *A, int lda, const unsigned short *W, int ldw, const float *bias, int64_t M, int N,
         int K, float *Cf, int ldc, unsigned short *Cb, int ldcb, const float *Zin, int n_valid, hipStream_t s,
         const unsigned long long *live = nullptr)
{
    hipLaunchKernelGGL(k_gemm_nt<EPI>, dim3((unsigned)(N / 64), (unsigned)(M / 64)), dim3(256), 0, s, A, lda, W,
                       ldw, bias, K, Cf, ldc, Cb, ldcb, Zin, n_valid, live);
    return (int)hipGetLastError();
}

}  // namespace

int mlp_gemm_plain(const unsigned short *A, int lda, const unsigned short *W, int ldw, int64_t M, int N, int K,
                   float *C, int ldc, hipStream_t s)
{
    return gemm<EPI_PLAIN>(A, lda, W, ldw, nullptr, M, N, K, C, ldc, nullptr, 0, nullptr, N, s);
}

int mlp_refresh_shadow(const MlpDevice &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_shadow, dim3(blocks_for((int64_t)kHidden * kHidden)), dim3(256), 0, s, d.params, d.w2,
                       d.w2t, d.w3, d.w3t, d.w4, d.w4t, d.w5);
    return (int)hipGetLastError();
}

// Forward pass for `rows` rows (multiple of 64).  train: keep z1..z4 (f32) for the backward pass.
// live (device, optional): only the first *live rows (rounded up to 64) are computed.
int mlp_forward(const MlpDevice &d, const MlpBuffers &b, const float *x, int64_t rows, float *y, bool train,
                hipStream_t s, const unsigned long long *live)
{
    int e;
    hipLaunchKernelGGL(k_layer1, dim3(blocks_for(rows * kHidden)), dim3(256), 0, s, x, d.params + kOffW1,
                       d.params + kOffB1, rows, train ? b.z[0] : nullptr, b.a[0], live);
    if ((e = (int)hipGetLastError())) return e;
    const unsigned short *w[3] = {d.w2, d.w3, d.w4};
    const int boff[3] = {kOffB2, kOffB3, kOffB4};
    for (int l = 0; l < 3; ++l) {
        if (train)
            e = gemm<EPI_BIAS_Z_GELU>(b.a[l], kHidden, w[l], kHidden, d.params + boff[l], rows, kHidden, kHidden,
                                      b.z[l + 1], kHidden, b.a[l + 1], kHidden, nullptr, kHidden, s, live);
        else
            e = gemm<EPI_BIAS_GELU>(b.a[l], kHidden, w[l], kHidden, d.params + boff[l], rows, kHidden, kHidden,
                                    nullptr, kHidden, b.a[l + 1], kHidden, nullptr, kHidden, s, live);
        if (e) return e;
    }
    return gemm<EPI_BIAS_OUT>(b.a[3], kHidden, d.w5, kHidden, d.params + kOffB5, rows, kOutPad, kHidden, y, kOut,
                              nullptr, 0, nullptr, kOut, s, live);
}

// Backward pass after a training forward: MSE gradients of all parameters into d.grad;
// per-block loss sums into b.loss_part (blocks_for(rows * 6) of them).
int mlp_backward(const MlpDevice &d, const MlpBuffers &b, const float *x, const float *t, int64_t rows,
                 const float *y, hipStream_t s)
{
    int e;
    float *dz = b.dz, *dz2 = b.dz2;
    unsigned short *dzb = b.dzb, *dzb2 = b.dzb2;
    hipLaunchKernelGGL(k_out_error, dim3(blocks_for(rows * kOut)), dim3(256), 0, s, y, t, rows, b.dy, b.loss_part);
    if ((e = (int)hipGetLastError())) return e;
    // W5 [6][256] = dy^T a4, b5 = column sums of dy
    if ((e = wide_reduce(b.a[3], true, rows, b.dy, kOut, false, true, true, d.grad + kOffW5, nullptr,
                         d.grad + kOffB5, b.part, s)))
        return e;
    // error into layer 4
    hipLaunchKernelGGL(k_out_back, dim3(blocks_for(rows * kHidden)), dim3(256), 0, s, b.dy, d.params + kOffW5,
                       b.z[3], rows, dz, dzb);
    if ((e = (int)hipGetLastError())) return e;
    const int woff[3] = {kOffW2, kOffW3, kOffW4}, boff[3] = {kOffB2, kOffB3, kOffB4};
    const unsigned short *wt[3] = {d.w2t, d.w3t, d.w4t};
    for (int l = 2; l >= 0; --l) {  // hidden layer l + 2: input a[l], pre-activation z[l + 1]
        // dW = dz^T a_prev: NT product of the transposes (K = rows)
        hipLaunchKernelGGL(k_transpose, dim3(kHidden / 32, (unsigned)((rows + 31) / 32)), dim3(256), 0, s, dzb,
                           rows, kHidden, b.t0);
        hipLaunchKernelGGL(k_transpose, dim3(kHidden / 32, (unsigned)((rows + 31) / 32)), dim3(256), 0, s, b.a[l],
                           rows, kHidden, b.t1);
        if ((e = (int)hipGetLastError())) return e;
        // split over the rows (K) so that the 16 output tiles become 16 x nsplit blocks
        int nsplit = 16;
        while (nsplit > 1 && (rows % (32 * nsplit) != 0 || rows / nsplit < 128)) nsplit /= 2;
        hipLaunchKernelGGL(k_gemm_nt<EPI_PLAIN>, dim3(kHidden / 64, kHidden / 64, (unsigned)nsplit), dim3(256), 0,
                           s, (const unsigned short *)b.t0, (int)rows, (const unsigned short *)b.t1, (int)rows,
                           (const float *)nullptr, (int)(rows / nsplit), b.part, kHidden, (unsigned short *)nullptr,
                           0, (const float *)nullptr, kHidden, (const unsigned long long *)nullptr);
        hipLaunchKernelGGL(k_split_sum, dim3(blocks_for((int64_t)kHidden * kHidden)), dim3(256), 0, s,
                           (const float *)b.part, nsplit, (int64_t)kHidden * kHidden, d.grad + woff[l]);
        if ((e = (int)hipGetLastError())) return e;
        if ((e = wide_reduce(dz, false, rows, nullptr, 0, true, false, false, nullptr, d.grad + boff[l], nullptr,
                             b.part2, s)))
            return e;
        // error into the layer below: dz_below = (dz W) * g'(z_below)
        if ((e = gemm<EPI_GELU_BACK>(dzb, kHidden, wt[l], kHidden, nullptr, rows, kHidden, kHidden, dz2,
                                     kHidden, dzb2, kHidden, b.z[l], kHidden, s)))
            return e;
        std::swap(dz, dz2);
        std::swap(dzb, dzb2);
    }
    // W1 [256][6] = dz1^T x, b1 = column sums of dz1 (both wide)
    return wide_reduce(dz, false, rows, x, kIn, true, false, false, d.grad + kOffW1, d.grad + kOffB1, nullptr, b.part,
                       s);
}

int mlp_infer(const MlpDevice &d, const float *x, int64_t rows, float *y, hipStream_t s,
              const unsigned long long *live)
{
    if (rows <= 0) return 0;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((rows + kFuseRows - 1) / kFuseRows)), dim3(64 * kFuseWaves), 0, s,
                       x, rows,
                       live, (const float *)d.params, (const unsigned short *)d.w2, (const unsigned short *)d.w3,
                       (const unsigned short *)d.w4, (const unsigned short *)d.w5, y);
    return (int)hipGetLastError();
}

int mlp_loss_mean(const MlpBuffers &b, int64_t rows, float *out, hipStream_t s, const int *step)
{
    hipLaunchKernelGGL(k_loss_mean, dim3(1), dim3(256), 0, s, (const float *)b.loss_part,
                       (int)blocks_for(rows * kOut), 1.0f / (float)(rows * kOut), out, step);
    return (int)hipGetLastError();
}

int mlp_adam_sched(const MlpDevice &d, const int *step, int total, float lr_max, float lr_min, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam_sched, dim3(blocks_for(kParams)), dim3(256), 0, s, d.params, d.grad, d.m, d.v,
                       (int64_t)kParams, step, total, lr_max, lr_min, 0.9f, 0.999f, 1e-8f);
    int e = (int)hipGetLastError();
    if (e) return e;
    return mlp_refresh_shadow(d, s);
}

int mlp_step_advance(int *step, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step);
    return (int)hipGetLastError();
}

int mlp_adam(const MlpDevice &d, float lr, int step, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(kParams)), dim3(256), 0, s, d.params, d.grad, d.m, d.v,
                       (int64_t)kParams, lr, b1, b2, 1e-8f, c1, c2);
    int e = (int)hipGetLastError();
    if (e) return e;
    return mlp_refresh_shadow(d, s);
}

}  // namespace pbr
