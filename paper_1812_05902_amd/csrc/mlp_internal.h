// Internal interface of the ray-surrogate network kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace pbr {

constexpr int kIn = 6, kHidden = 256, kOut = 6;
constexpr int kOutPad = 64;  // output layer padded to the 64-wide product tile (zero rows)

// Flat FP32 parameter layout: W1 [256][6], b1, W2 [256][256], b2, W3, b3, W4, b4, W5 [6][256], b5.
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kIn;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden * kHidden;
constexpr int kOffW4 = kOffB3 + kHidden;
constexpr int kOffB4 = kOffW4 + kHidden * kHidden;
constexpr int kOffW5 = kOffB4 + kHidden;
constexpr int kOffB5 = kOffW5 + kOut * kHidden;
constexpr int kParams = kOffB5 + kOut;
static_assert(kParams == 200710, "parameter count");

enum : int { EPI_PLAIN = 0, EPI_BIAS_GELU = 1, EPI_BIAS_Z_GELU = 2, EPI_BIAS_OUT = 3, EPI_GELU_BACK = 4 };

// Parameters, gradients, Adam moments (FP32) and the bf16 copies read by the matrix products.
struct MlpDevice {
    float *params, *grad, *m, *v;
    unsigned short *w2, *w2t, *w3, *w3t, *w4, *w4t;  // [256][256] and transposed
    unsigned short *w5;                              // [64][256], rows 6..63 zero
};

// Per-batch buffers for up to rows_cap rows (a multiple of 64).
struct MlpBuffers {
    int64_t rows_cap;
    float *z[4];            // pre-activations of layers 1..4 (f32)
    unsigned short *a[4];   // activations of layers 1..4 (bf16)
    float *dy;              // [rows][6]
    float *dz, *dz2;        // [rows][256] f32
    unsigned short *dzb, *dzb2, *t0, *t1;
    float *loss_part;       // ceil(rows * 6 / 256) partial sums
    float *part, *part2;    // 16 x 256 x 256 floats each: split-K slices and row-block partial sums
};

int mlp_refresh_shadow(const MlpDevice &d, hipStream_t s);
int mlp_forward(const MlpDevice &d, const MlpBuffers &b, const float *x, int64_t rows, float *y, bool train,
                hipStream_t s, const unsigned long long *live = nullptr);
int mlp_backward(const MlpDevice &d, const MlpBuffers &b, const float *x, const float *t, int64_t rows,
                 const float *y, hipStream_t s);
// Inference forward pass in one launch (activations in LDS), any row count; live (device,
// optional) caps the rows computed.  Same roundings as mlp_forward (the products may sum in
// another order inside the matrix cores).
int mlp_infer(const MlpDevice &d, const float *x, int64_t rows, float *y, hipStream_t s,
              const unsigned long long *live = nullptr);
// After mlp_backward: *out (device) = mean squared error of that batch (out[*step] if step given).
int mlp_loss_mean(const MlpBuffers &b, int64_t rows, float *out, hipStream_t s, const int *step = nullptr);
// Adam step with t = *step + 1 and the cosine learning rate of step *step out of total (device step
// counter, so that one captured graph serves every step), then the bf16 copies.
int mlp_adam_sched(const MlpDevice &d, const int *step, int total, float lr_max, float lr_min, hipStream_t s);
int mlp_step_advance(int *step, hipStream_t s);
int mlp_adam(const MlpDevice &d, float lr, int step, hipStream_t s);
// C[M][N] = A[M][K] W[N][K]^T in f32 (bf16 operands); M, N multiples of 64, K of 32.
int mlp_gemm_plain(const unsigned short *A, int lda, const unsigned short *W, int ldw, int64_t M, int N, int K,
                   float *C, int ldc, hipStream_t s);

}  // namespace pbr
