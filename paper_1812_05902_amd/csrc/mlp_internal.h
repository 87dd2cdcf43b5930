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

// Parameters, gradients, Adam moments (FP32) and the bf16 copies read by the matrix products.
struct MlpDevice {
    float *params, *grad, *m, *v;
    unsigned short *w2, *w2t, *w3, *w3t, *w4, *w4t;  // [256][256] and transposed
    unsigned short *w5;                              // [64][256], rows 6..63 zero
};

// Buffers of a training step for batches of up to rows_cap rows (a multiple of 64).
constexpr int kTrainPartStride = 4224;  // floats per row-block record (row sums of the small gradients)
constexpr int kTrainBlockRows = 16;     // rows per block of the training pass's row kernel
constexpr int kMaxDwSplits = 16;        // row slices of the weight-gradient products
struct MlpTrain {
    int64_t rows_cap;
    unsigned short *aT[3];   // activations a1, a2, a3 (bf16) transposed: [256][rows_cap]
    unsigned short *dzT[3];  // errors dz2, dz3, dz4 (bf16) transposed: [256][rows_cap]
    float *zbuf;             // pre-activations of layers 1..4: [4][rows_cap][256] f32
    float *rowpart;          // [rows_cap / kTrainBlockRows][kTrainPartStride]
    float *rowsum;           // [groups of 16 row blocks][kTrainPartStride]
    float *dwpart;           // [3][kMaxDwSplits][256][256]
};

int mlp_refresh_shadow(const MlpDevice &d, hipStream_t s);
// Inference forward pass in one launch (activations in LDS), any row count; live (device,
// optional) caps the rows computed.
int mlp_infer(const MlpDevice &d, const float *x, int64_t rows, float *y, hipStream_t s,
              const unsigned long long *live = nullptr);
// One training step on x, t ([rows][6] device, rows a multiple of 64 up to rows_cap): forward,
// mean squared error, gradients of every parameter into d.grad, and
//   mode 0: nothing more (loss_out[0] = the loss);
//   mode 1: Adam with learning rate lr at step number `step` (1-based), bf16 copies refreshed;
//   mode 2: Adam at step *step_dev + 1 with the cosine learning rate from lr_max (step 0) to lr_min
//           (step total - 1), the counter advanced, loss_out[*step_dev] = the loss (one captured
//           graph serves every step).
int mlp_train_step(const MlpDevice &d, const MlpTrain &tb, const float *x, const float *t, int64_t rows, int mode,
                   float lr, int step, int *step_dev, int total, float lr_max, float lr_min, float *loss_out,
                   hipStream_t s);

}  // namespace pbr
