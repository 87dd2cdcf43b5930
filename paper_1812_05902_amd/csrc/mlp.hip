// Kernels of the ray-surrogate network 6 -> 256 -> 256 -> 256 -> 256 -> 6 (GELU, tanh form):
// the input layer in FP32 (entry positions need more than bfloat16's 8 bits), the three hidden
// 256 x 256 layers and the output layer as bfloat16 matrix products on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation); a training step in three kernels (the forward
// pass, the loss and the back-propagated errors of 16 rows per block; the weight-gradient
// products; the fixed-order gradient sums, Adam on the FP32 master weights and the bfloat16
// shadow copies).
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


// ---------------------------------------------------------------- training step
//
// One step over a batch of `rows` rows (a multiple of 64) in three launches:
//   k_train_rows   one block per 16 rows: layer 1 .. output forward with every pre-activation parked
//                  in an L2-resident buffer, the loss and dL/dy, the back-propagated errors down to
//                  layer 1, and per block the row sums the small gradients need (biases, W1, W5, b5,
//                  the loss), the small ones as FP32 matrix-core products;
//                  writes the bf16 activations a1..a3 and errors dz2..dz4 transposed ([unit][row],
//                  the layout the weight-gradient products read);
//   k_train_dw     dW_l = bf16(dz_l)^T a_(l-1) for the three hidden layers, the rows split into S
//                  slices (partial sums per slice);
//   k_train_update one thread per parameter: its gradient summed over the slices / row blocks in a
//                  fixed order, then Adam and the bf16 shadow copies (or the gradient only).
// The roundings are those of the unfused formulation: bf16 weights of layers 2-5, bf16 activations
// and bf16 errors feeding the matrix products, FP32 everywhere else (layer 1, pre-activations,
// dL/dy, the error of layer 4 from the FP32 W5, biases, all sums).

// Per-block record of row sums written by k_train_rows (floats).
constexpr int kRpB = 0;                         // b1..b4 sums [4][256], layer l at (l - 1) * 256
constexpr int kRpW1 = 4 * kHidden;              // W1 [256][6]
constexpr int kRpW5 = kRpW1 + kHidden * kIn;    // W5 [6][256]
constexpr int kRpB5 = kRpW5 + kOut * kHidden;   // b5 [6]
constexpr int kRpLoss = kRpB5 + kOut;           // sum of squared errors
static_assert(kRpLoss < kTrainPartStride, "row-block record");

constexpr int kTrRows = kTrainBlockRows;  // rows per k_train_rows block; eight waves own 32 units each
constexpr int kTrTiles = kTrRows / 16;     // 16-row tiles per block

// Accumulators of a kTrRows-row x 32-unit slab: [unit tile j][row tile i], lane (r, kg) holding units
// 16 j + 4 kg + t of row 16 i + r (the transposed-product layout of k_mlp_infer).
struct Slab {
    floatx4 v[2][kTrTiles];
};

// The wave's 32 rows of a [256][256] bf16 weight matrix (output units wave * 32 .. + 31, k
// contiguous) as the A operands of all eight k steps of a slab product, and the matching biases
// (zero without a bias).
struct WFrag {
    bf16x8 f[8][2];
    floatx4 b[2];
};

__device__ __forceinline__ void load_wfrag(WFrag &w, const unsigned short *__restrict__ W,
                                           const float *__restrict__ bias, int wave, int r, int kg)
{
    const unsigned short *Wr = W + (size_t)(wave * 32 + r) * kHidden + 8 * kg;
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j) w.f[k][j] = *(const bf16x8 *)(Wr + j * 16 * kHidden + 32 * k);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        w.b[j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        if (bias) {
            const float4 b4 = *(const float4 *)(bias + wave * 32 + 16 * j + 4 * kg);
            w.b[j] = floatx4{b4.x, b4.y, b4.z, b4.w};
        }
    }
}

// Z^T = W A^T (+ bias) over K = 256 for this wave's 32 units and the kTrRows rows in `act` (LDS
// [row][unit] bf16), with the weights already in `w`.
__device__ __forceinline__ void slab_product(Slab &acc, const WFrag &w, const unsigned short *act, int r, int kg)
{
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < kTrTiles; ++i) acc.v[j][i] = w.b[j];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
        for (int i = 0; i < kTrTiles; ++i) {
            const bf16x8 fa = *(const bf16x8 *)(act + (16 * i + r) * kActStride + 8 * kg + 32 * k);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc.v[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.f[k][j], fa, acc.v[j][i], 0, 0, 0);
        }
    }
}

// bf16 values of a slab (of g applied to it when GELU) into LDS [row][unit] and, when T is given,
// into T [unit][ldt] (the transposed layout of the weight-gradient products).  Within each block
// of kTrRows rows, T holds row 16 i + r at column kTrTiles r + i, so that a lane's row tiles are
// one store; the weight-gradient products sum over rows and read both of their operands in this
// same order, so the permutation only reorders the terms of their sums.
template <bool GELU>
__device__ __forceinline__ void slab_store(const Slab &v, unsigned short *act, unsigned short *__restrict__ T,
                                           int64_t ldt, int64_t row0, int wave, int r, int kg)
{
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        unsigned short b[kTrTiles][4];  // [row tile i][unit t]
        const int u = wave * 32 + 16 * j + 4 * kg;
#pragma unroll
        for (int i = 0; i < kTrTiles; ++i) {
#pragma unroll
            for (int t = 0; t < 4; ++t) b[i][t] = bf16_bits(GELU ? gelu(v.v[j][i][t]) : v.v[j][i][t]);
            uint2 w;
            w.x = (unsigned)b[i][0] | ((unsigned)b[i][1] << 16);
            w.y = (unsigned)b[i][2] | ((unsigned)b[i][3] << 16);
            *(uint2 *)(act + (16 * i + r) * kActStride + u) = w;
        }
        if (T) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                unsigned short *d = T + (size_t)(u + t) * ldt + row0 + kTrTiles * r;
                if (kTrTiles == 4) {
                    uint2 w;
                    w.x = (unsigned)b[0][t] | ((unsigned)b[1 % kTrTiles][t] << 16);
                    w.y = (unsigned)b[2 % kTrTiles][t] | ((unsigned)b[3 % kTrTiles][t] << 16);
                    *(uint2 *)d = w;
                } else if (kTrTiles == 2) {
                    *(unsigned *)d = (unsigned)b[0][t] | ((unsigned)b[1 % kTrTiles][t] << 16);
                } else {
                    *d = b[0][t];
                }
            }
        }
    }
}

// Sum over the 16 lanes of a DPP row (lanes r = 0..15 of one kg): xor-1 and xor-2 exchanges inside
// each quad, then the half-row and row mirrors; every lane ends with the same value as a
// butterfly of xor shuffles gives.
__device__ __forceinline__ float row16_sum(float s)
{
    s += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    s += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    s += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), 0x141, 0xF, 0xF, false));  // row_half_mirror
    s += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), 0x140, 0xF, 0xF, false));  // row_mirror
    return s;
}

// Sum of a slab over its kTrRows rows, per unit: lanes r = 0 of each kg end with the sums of units
// 16 j + 4 kg + t; written to out[wave * 32 + unit].
__device__ __forceinline__ void slab_row_sums(const Slab &v, float *__restrict__ out, int wave, int r, int kg)
{
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            // the block's row tiles added pairwise in a fixed tree, then the 16 rows of a tile
            float a = v.v[j][0][t];
            if (kTrTiles == 2) a = v.v[j][0][t] + v.v[j][1 % kTrTiles][t];
            if (kTrTiles == 4)
                a = (v.v[j][0][t] + v.v[j][1 % kTrTiles][t]) + (v.v[j][2 % kTrTiles][t] + v.v[j][3 % kTrTiles][t]);
            const float s = row16_sum(a);
            if (r == 0) out[wave * 32 + 16 * j + 4 * kg + t] = s;
        }
}

// LDS of k_train_rows: two bf16 [64][kActStride] activation / error buffers, later reused for
// layer 1's FP32 error as [unit][kDz1Stride] (the stride keeps the W1 product's reads free of bank
// conflicts).
constexpr int kDz1Stride = kTrRows + 4;
constexpr int kK1ActBytes = 2 * kTrRows * kActStride * 2;
constexpr int kK1LdsBytes = kK1ActBytes > kHidden * kDz1Stride * 4 ? kK1ActBytes : kHidden * kDz1Stride * 4;

// Every global load is issued as early as its registers allow: vector memory operations complete
// in issue order, so a load queued behind another layer's stores or weight fetch waits for them.
__global__ void __launch_bounds__(512, 1) k_train_rows(const float *__restrict__ params,
                                                       const unsigned short *__restrict__ w2,
                                                       const unsigned short *__restrict__ w3,
                                                       const unsigned short *__restrict__ w4,
                                                       const unsigned short *__restrict__ w2t,
                                                       const unsigned short *__restrict__ w3t,
                                                       const unsigned short *__restrict__ w4t,
                                                       const unsigned short *__restrict__ w5,
                                                       const float *__restrict__ x, const float *__restrict__ tgt,
                                                       int64_t rows, int64_t ldt, MlpTrain tb)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[kK1LdsBytes];
    __shared__ float xs[kTrRows * kIn], ts[kTrRows * kIn], dys[kTrRows * kOut];
    __shared__ float red[kTrRows];
    auto act = [&](int b) { return (unsigned short *)lds + b * (kTrRows * kActStride); };
    const int64_t row0 = (int64_t)blockIdx.x * kTrRows;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kg = lane >> 4;
    float *rp = tb.rowpart + (size_t)blockIdx.x * kTrainPartStride;
    // pre-activations of layers 1..3, parked in L2-resident memory until the backward pass needs
    // them (each lane reads back exactly what it wrote); layer 4's stay in registers
    auto zp = [&](int l, int j, int i) {
        return tb.zbuf + ((size_t)l * ldt + row0 + 16 * i + r) * kHidden + wave * 32 + 16 * j + 4 * kg;
    };
    auto park = [&](const Slab &v, int l) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < kTrTiles; ++i) *(floatx4 *)zp(l, j, i) = v.v[j][i];
    };
    auto unpark = [&](Slab &v, int l) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < kTrTiles; ++i) v.v[j][i] = *(const floatx4 *)zp(l, j, i);
    };
    // inputs, targets and layer 1's parameters first, then the weights of layer 2
    float xv = 0.0f, tv = 0.0f;
    if (threadIdx.x < kTrRows * kIn) {
        xv = x[row0 * kIn + threadIdx.x];
        tv = tgt[row0 * kIn + threadIdx.x];
    }
    float w1a[2][2];
    floatx4 b1[2];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = 4 * kk + kg;
            w1a[kk][j] = k < kIn ? params[kOffW1 + (wave * 32 + 16 * j + r) * kIn + k] : 0.0f;
        }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float4 b4 = *(const float4 *)(params + kOffB1 + wave * 32 + 16 * j + 4 * kg);
        b1[j] = floatx4{b4.x, b4.y, b4.z, b4.w};
    }
    WFrag fw;
    load_wfrag(fw, w2, params + kOffB2, wave, r, kg);
    if (threadIdx.x < kTrRows * kIn) {
        xs[threadIdx.x] = xv;
        ts[threadIdx.x] = tv;
    }
    __syncthreads();
    {   // layer 1 in FP32 on the matrix cores (v_mfma_f32_16x16x4_f32, K = 6 padded to 8)
        Slab z;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < kTrTiles; ++i) z.v[j][i] = b1[j];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int k = 4 * kk + kg;
#pragma unroll
            for (int i = 0; i < kTrTiles; ++i) {
                const float xb = k < kIn ? xs[(16 * i + r) * kIn + k] : 0.0f;
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    z.v[j][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1a[kk][j], xb, z.v[j][i], 0, 0, 0);
            }
        }
        // a1 = bf16(g(z1)) into act(0) (the input of layer 2) and transposed for dW2
        park(z, 0);
        slab_store<true>(z, act(0), tb.aT[0], ldt, row0, wave, r, kg);
    }
    __syncthreads();
    // layers 2 and 3: z = a W^T + b, a = bf16(g(z)); inputs in act(l & 1), outputs to act((l + 1) & 1)
#pragma unroll 1
    for (int l = 0; l < 2; ++l) {
        Slab z;
        slab_product(z, fw, act(l & 1), r, kg);
        load_wfrag(fw, l == 0 ? w3 : w4, params + (l == 0 ? kOffB3 : kOffB4), wave, r, kg);
        park(z, l + 1);
        slab_store<true>(z, act((l + 1) & 1), tb.aT[l + 1], ldt, row0, wave, r, kg);
        __syncthreads();
    }
    // layer 4 (input a3 in act(0), output a4 to act(1)); then the loads of the output layer and of
    // dz4 (the bf16 W5 fragments, FP32 W5 and b5) ahead of the first backward weights, W4^T
    Slab dz;  // z4, then dz4
    slab_product(dz, fw, act(0), r, kg);
    bf16x8 f5[8];
    float b5v[4];
    if (wave < kTrTiles) {
#pragma unroll
        for (int k = 0; k < 8; ++k) f5[k] = *(const bf16x8 *)(w5 + (size_t)r * kHidden + 8 * kg + 32 * k);
#pragma unroll
        for (int t = 0; t < 4; ++t) b5v[t] = (kg < 2 && 4 * kg + t < kOut) ? params[kOffB5 + 4 * kg + t] : 0.0f;
    }
    float w5a[2][2];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int o = 4 * kk + kg;
            w5a[kk][j] = o < kOut ? params[kOffW5 + o * kHidden + wave * 32 + 16 * j + r] : 0.0f;
        }
    load_wfrag(fw, w4t, nullptr, wave, r, kg);
    slab_store<true>(dz, act(1), nullptr, ldt, row0, wave, r, kg);
    __syncthreads();
    // output layer (16 padded outputs x 16 rows per wave, waves 0..3), loss, dL/dy
    if (wave < kTrTiles) {
        floatx4 acc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bf16x8 fa = *(const bf16x8 *)(act(1) + (16 * wave + r) * kActStride + 8 * kg + 32 * k);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f5[k], fa, acc, 0, 0, 0);
        }
        const int m = 16 * wave + r;
        const float scale = 2.0f / (float)(rows * kOut);
        float se = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int o = 4 * kg + t;
            if (kg < 2 && o < kOut) {
                const float d = (acc[t] + b5v[t]) - ts[m * kIn + o];
                dys[m * kOut + o] = scale * d;
                se += d * d;
            }
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) se += __shfl_xor(se, o, 64);
        if (lane == 0) red[wave] = se;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float l = red[0];
        if (kTrTiles == 2) l = red[0] + red[1];
        if (kTrTiles == 4) l = (red[0] + red[1]) + (red[2] + red[3]);
        rp[kRpLoss] = l;
    }
    Slab zn;  // the next backward layer's pre-activations, z3
    unpark(zn, 2);
    {   // W5 and b5 gradients, C[o][u] = sum over rows of dy[m][o] a4[m][u] (a4 as stored in bf16),
        // on v_mfma_f32_16x16x4_f32 with o padded to 16; b5 as the product with a column of ones
        floatx4 g[2] = {floatx4{0.0f, 0.0f, 0.0f, 0.0f}, floatx4{0.0f, 0.0f, 0.0f, 0.0f}};
        floatx4 gb = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s4 = 0; s4 < kTrRows; s4 += 4) {
            const int m = s4 + kg;
            const float a = r < kOut ? dys[m * kOut + r] : 0.0f;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const float b = __uint_as_float((unsigned)act(1)[m * kActStride + wave * 32 + 16 * j + r] << 16);
                g[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, g[j], 0, 0, 0);
            }
            if (wave == 0) gb = __builtin_amdgcn_mfma_f32_16x16x4f32(a, r == 0 ? 1.0f : 0.0f, gb, 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int o = 4 * kg + t;
            if (o < kOut) {
#pragma unroll
                for (int j = 0; j < 2; ++j) rp[kRpW5 + o * kHidden + wave * 32 + 16 * j + r] = g[j][t];
                if (wave == 0 && r == 0) rp[kRpB5 + o] = gb[t];
            }
        }
    }
    {   // error of layer 4 from dy and the FP32 W5: dz4 = (dy W5) g'(z4), the product on
        // v_mfma_f32_16x16x4_f32 (units x rows, K = 6 outputs padded to 8)
        Slab da;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < kTrTiles; ++i) da.v[j][i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int o = 4 * kk + kg;
#pragma unroll
            for (int i = 0; i < kTrTiles; ++i) {
                const float yb = o < kOut ? dys[(16 * i + r) * kOut + o] : 0.0f;
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    da.v[j][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(w5a[kk][j], yb, da.v[j][i], 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < kTrTiles; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) dz.v[j][i][t] = da.v[j][i][t] * gelu_grad(dz.v[j][i][t]);
    }
    slab_row_sums(dz, rp + kRpB + 3 * kHidden, wave, r, kg);
    slab_store<false>(dz, act(0), tb.dzT[2], ldt, row0, wave, r, kg);  // a3 in act(0) is no longer read
    __syncthreads();
    // errors of layers 3, 2, 1: dz_(l+1) = (bf16(dz_(l+2)) W_(l+2)) g'(z_(l+1)), with W^T rows as the A
    // operand; layer l + 2's error in act(l & 1); the next weights and pre-activations are fetched
    // before this layer's stores
#pragma unroll 1
    for (int l = 2; l >= 0; --l) {
        const Slab zl = zn;
        slab_product(dz, fw, act(l & 1), r, kg);
        if (l > 0) {
            load_wfrag(fw, l == 2 ? w3t : w2t, nullptr, wave, r, kg);
            unpark(zn, l - 1);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < kTrTiles; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) dz.v[j][i][t] *= gelu_grad(zl.v[j][i][t]);
        slab_row_sums(dz, rp + kRpB + l * kHidden, wave, r, kg);
        if (l > 0) slab_store<false>(dz, act((l + 1) & 1), tb.dzT[l - 1], ldt, row0, wave, r, kg);
        __syncthreads();
    }
    // W1 gradient, C[k][u] = sum over rows of x[m][k] dz1[m][u] in FP32 on v_mfma_f32_16x16x4_f32
    // (k padded to 16): dz1 goes through LDS as [unit][row] to put the rows on the K operand lanes
    float *dzf = (float *)lds;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < kTrTiles; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) dzf[(wave * 32 + 16 * j + 4 * kg + t) * kDz1Stride + 16 * i + r] = dz.v[j][i][t];
    __syncthreads();
    floatx4 g1[2] = {floatx4{0.0f, 0.0f, 0.0f, 0.0f}, floatx4{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
    for (int s4 = 0; s4 < kTrRows; s4 += 4) {
        const int m = s4 + kg;
        const float a = r < kIn ? xs[m * kIn + r] : 0.0f;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            g1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, dzf[(wave * 32 + 16 * j + r) * kDz1Stride + m], g1[j], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = 4 * kg + t;
        if (k < kIn) {
#pragma unroll
            for (int j = 0; j < 2; ++j) rp[kRpW1 + (wave * 32 + 16 * j + r) * kIn + k] = g1[j][t];
        }
    }
}

// Weight-gradient products of the three hidden layers, rows split into slices:
// part[l][z][n][k] = sum over rows m of slice z of dzT_l[n][m] aT_(l-1)[k][m] (both bf16,
// [unit][ld] with the rows contiguous).  Grid (4, 4, 3 * nsplit + extra), 64 x 64 output tiles, four
// waves of 32 x 32.  Block (0, 0, 0) also advances the step counter when one is given.  The blocks
// of the extra z layers each add up a group of kRowGroup row-block records of k_train_rows, in
// block order, into one group record (so that the update adds a few group records per parameter
// instead of every row block's).
constexpr int kRowGroup = 16;
constexpr int kRowChunks = (kRpLoss + 256) / 256;  // 256-column chunks of a record

__global__ void __launch_bounds__(256) k_train_dw(MlpTrain tb, int64_t ldt, int64_t chunk, int nsplit, int nblocks,
                                                  int *step_advance)
{
    if ((int)blockIdx.z >= 3 * nsplit) {
        // block e: record columns 256 (e mod kRowChunks) .. + 255 of group e / kRowChunks; the
        // group's loads are all issued before the sum
        const int e = ((int)blockIdx.z - 3 * nsplit) * 16 + (int)blockIdx.y * 4 + (int)blockIdx.x;
        const int g = e / kRowChunks, c = (e % kRowChunks) * 256 + (int)threadIdx.x;
        const int b0 = g * kRowGroup;
        if (b0 >= nblocks || c > kRpLoss) return;
        float v[kRowGroup];
#pragma unroll
        for (int b = 0; b < kRowGroup; ++b)
            v[b] = b0 + b < nblocks ? tb.rowpart[(size_t)(b0 + b) * kTrainPartStride + c] : 0.0f;
        float s = v[0];
#pragma unroll
        for (int b = 1; b < kRowGroup; ++b) s += v[b];
        tb.rowsum[(size_t)g * kTrainPartStride + c] = s;
        return;
    }
    const int l = blockIdx.z / nsplit, z = blockIdx.z % nsplit;
    if (step_advance && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *step_advance += 1;
    const unsigned short *A = tb.dzT[l] + (size_t)z * chunk;
    const unsigned short *W = tb.aT[l] + (size_t)z * chunk;
    float *C = tb.dwpart + ((size_t)l * kMaxDwSplits + z) * kHidden * kHidden;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;  // n (output unit of dz)
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;   // k (input unit)
    const int r = lane & 15, kg = lane >> 4;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const unsigned short *a0 = A + (size_t)(m0 + r) * ldt + 8 * kg;
    const unsigned short *a1 = A + (size_t)(m0 + 16 + r) * ldt + 8 * kg;
    const unsigned short *b0 = W + (size_t)(n0 + r) * ldt + 8 * kg;
    const unsigned short *b1 = W + (size_t)(n0 + 16 + r) * ldt + 8 * kg;
    // chunk is a multiple of 64: two k steps per iteration, the next two loaded ahead
    bf16x8 f[4], g[4];
    f[0] = *(const bf16x8 *)a0; f[1] = *(const bf16x8 *)a1; f[2] = *(const bf16x8 *)b0; f[3] = *(const bf16x8 *)b1;
    g[0] = *(const bf16x8 *)(a0 + 32); g[1] = *(const bf16x8 *)(a1 + 32);
    g[2] = *(const bf16x8 *)(b0 + 32); g[3] = *(const bf16x8 *)(b1 + 32);
    for (int64_t k0 = 0; k0 < chunk; k0 += 64) {
        bf16x8 fn[4], gn[4];
        const bool more = k0 + 64 < chunk;
        if (more) {
            fn[0] = *(const bf16x8 *)(a0 + k0 + 64); fn[1] = *(const bf16x8 *)(a1 + k0 + 64);
            fn[2] = *(const bf16x8 *)(b0 + k0 + 64); fn[3] = *(const bf16x8 *)(b1 + k0 + 64);
            gn[0] = *(const bf16x8 *)(a0 + k0 + 96); gn[1] = *(const bf16x8 *)(a1 + k0 + 96);
            gn[2] = *(const bf16x8 *)(b0 + k0 + 96); gn[3] = *(const bf16x8 *)(b1 + k0 + 96);
        }
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[0], f[2], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[0], f[3], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[1], f[2], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[1], f[3], acc[1][1], 0, 0, 0);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g[0], g[2], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g[0], g[3], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g[1], g[2], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g[1], g[3], acc[1][1], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int c = 0; c < 4; ++c) { f[c] = fn[c]; g[c] = gn[c]; }
        }
    }
    // lane: rows 4 kg + t (n), column r (k) of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                C[(size_t)(m0 + 16 * i + 4 * kg + t) * kHidden + n0 + 16 * j + r] = acc[i][j][t];
}

// One thread per parameter: its gradient summed in a fixed order (hidden weights over the nsplit
// product slices, everything else over the row blocks), written to grad; mode 1: Adam with lr and
// step t given; mode 2: Adam with t = *step (advanced by k_train_dw) and the cosine learning rate
// of step t - 1 of `total`; modes 1, 2 then refresh the bf16 copies.  Thread 0 writes the batch's
// mean squared error to loss_out[0] (mode 2: loss_out[t - 1]).
__global__ void __launch_bounds__(256) k_train_update(MlpDevice d, MlpTrain tb, int ngroups, int nsplit,
                                                      float inv_count, int mode, float lr, int t_fixed,
                                                      const int *__restrict__ step, int total, float lr_max,
                                                      float lr_min, float *__restrict__ loss_out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    int t = t_fixed;
    if (mode == 2) t = *step;
    if (blockIdx.x == 0 && threadIdx.x < 64) {  // the loss: lane-strided partial sums, then a fixed tree
        float s = 0.0f;
        for (int b = threadIdx.x; b < ngroups; b += 64) s += tb.rowsum[(size_t)b * kTrainPartStride + kRpLoss];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (threadIdx.x == 0) loss_out[mode == 2 ? t - 1 : 0] = s * inv_count;
    }
    if (q >= kParams) return;
    float g = 0.0f;
    int wl = -1;  // hidden weight matrix 0..2 (W2..W4)
    int rec = -1; // offset in the row-block record
    if (q < kOffB1) rec = kRpW1 + (q - kOffW1);
    else if (q < kOffW2) rec = kRpB + (q - kOffB1);
    else if (q < kOffB2) wl = 0;
    else if (q < kOffW3) rec = kRpB + kHidden + (q - kOffB2);
    else if (q < kOffB3) wl = 1;
    else if (q < kOffW4) rec = kRpB + 2 * kHidden + (q - kOffB3);
    else if (q < kOffB4) wl = 2;
    else if (q < kOffW5) rec = kRpB + 3 * kHidden + (q - kOffB4);
    else if (q < kOffB5) rec = kRpW5 + (q - kOffW5);
    else rec = kRpB5 + (q - kOffB5);
    if (wl >= 0) {
        const int off = q - (wl == 0 ? kOffW2 : (wl == 1 ? kOffW3 : kOffW4));
        const float *p = tb.dwpart + (size_t)wl * kMaxDwSplits * kHidden * kHidden + off;
#pragma unroll 16
        for (int z = 0; z < nsplit; ++z) g += p[(size_t)z * kHidden * kHidden];
    } else {
        const float *p = tb.rowsum + rec;
        for (int b = 0; b < ngroups; ++b) g += p[(size_t)b * kTrainPartStride];
    }
    d.grad[q] = g;
    if (mode == 0) return;
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    float rate = lr;
    if (mode == 2) {
        const float ph = total > 1 ? (float)(t - 1) / (float)(total - 1) : 0.0f;
        rate = lr_min + 0.5f * (lr_max - lr_min) * (1.0f + cosf(3.14159265358979f * ph));
    }
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    const float mq = beta1 * d.m[q] + (1.0f - beta1) * g;
    const float vq = beta2 * d.v[q] + (1.0f - beta2) * g * g;
    d.m[q] = mq;
    d.v[q] = vq;
    const float pq = d.params[q] - rate * (mq / c1) / (sqrtf(vq / c2) + eps);
    d.params[q] = pq;
    if (wl >= 0) {
        const int off = q - (wl == 0 ? kOffW2 : (wl == 1 ? kOffW3 : kOffW4));
        const int o = off / kHidden, i = off % kHidden;
        unsigned short *w = wl == 0 ? d.w2 : (wl == 1 ? d.w3 : d.w4);
        unsigned short *wt = wl == 0 ? d.w2t : (wl == 1 ? d.w3t : d.w4t);
        const unsigned short b = bf16_bits(pq);
        w[off] = b;
        wt[i * kHidden + o] = b;
    } else if (q >= kOffW5 && q < kOffB5) {
        d.w5[q - kOffW5] = bf16_bits(pq);  // rows 6..63 of the padded copy stay zero
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Slices of the weight-gradient products: the largest divisor of rows / 64 not above
// kMaxDwSplits, so that every slice has the same multiple of 64 rows.
int dw_splits(int64_t rows)
{
    const int64_t g = rows / 64;
    int s = kMaxDwSplits;
    while (s > 1 && g % s != 0) --s;
    return s;
}

}  // namespace

int mlp_refresh_shadow(const MlpDevice &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_shadow, dim3(blocks_for((int64_t)kHidden * kHidden)), dim3(256), 0, s, d.params, d.w2,
                       d.w2t, d.w3, d.w3t, d.w4, d.w4t, d.w5);
    return (int)hipGetLastError();
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

int mlp_train_step(const MlpDevice &d, const MlpTrain &tb, const float *x, const float *t, int64_t rows, int mode,
                   float lr, int step, int *step_dev, int total, float lr_max, float lr_min, float *loss_out,
                   hipStream_t s)
{
    if (rows <= 0 || rows % 64 != 0 || rows > tb.rows_cap) return (int)hipErrorInvalidValue;
    const int nblocks = (int)(rows / kTrRows);
    hipLaunchKernelGGL(k_train_rows, dim3((unsigned)nblocks), dim3(512), 0, s, (const float *)d.params,
                       (const unsigned short *)d.w2, (const unsigned short *)d.w3, (const unsigned short *)d.w4,
                       (const unsigned short *)d.w2t, (const unsigned short *)d.w3t, (const unsigned short *)d.w4t,
                       (const unsigned short *)d.w5, x, t, rows, tb.rows_cap, tb);
    int e = (int)hipGetLastError();
    if (e) return e;
    const int ns = dw_splits(rows);
    const int ngroups = (nblocks + kRowGroup - 1) / kRowGroup;
    hipLaunchKernelGGL(k_train_dw, dim3(kHidden / 64, kHidden / 64, (unsigned)(3 * ns + (ngroups * kRowChunks + 15) / 16)),
                       dim3(256), 0, s, tb, tb.rows_cap, (int64_t)(rows / ns), ns, nblocks,
                       mode == 2 ? step_dev : (int *)nullptr);
    if ((e = (int)hipGetLastError())) return e;
    hipLaunchKernelGGL(k_train_update, dim3(blocks_for(kParams)), dim3(256), 0, s, d, tb, ngroups, ns,
                       1.0f / (float)(rows * kOut), mode, lr, step, (const int *)step_dev, total, lr_max, lr_min,
                       loss_out);
    return (int)hipGetLastError();
}

}  // namespace pbr
