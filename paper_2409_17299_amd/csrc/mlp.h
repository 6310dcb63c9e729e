// mlp.h -- the surrogate network of the emission inverse CDF: a 2 -> 64 -> 64
// -> 1 perceptron with SiLU activations.  Layer 2 runs on BF16 MFMA
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation: BF16 weights times the
// activations split into two bfloat16 parts; layers 1 and 3 run in FP32 on
// the vector ALUs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace sfqed {

constexpr int kH = 64;
// flat parameter order: W1[64][2], b1[64], W2[64][64] (out, in), b2[64], w3[64], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = 128;
constexpr int kOffW2 = 192;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;
constexpr int kMlpParams = kOffB3 + 1;  // 4417
// a partial-gradient row: the parameters, then the sum of squared residuals
constexpr int kGradRow = kMlpParams + 1;
constexpr int kMlpThreads = 256;        // four waves, each one 32-sample tile at a time

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Forms of the parameters the kernels read, written from the FP32 master copy.
// Feature slots: K-step s (0..3), lane half h (lane / 32), slot i (0..7) of a
// lane's 8-element MFMA operand hold feature
//   phi(s, h, i) = 32 (s / 2) + 16 (s % 2) + 8 (i / 4) + 4 h + i % 4,
// which is also the row of accumulator r = 8 (s % 2) + i of M-tile s / 2 in the
// 32x32 MFMA result layout.  Every layer of one lane therefore holds the same
// 32 features of one sample, and one layer's result is the next one's operand.
struct MlpPacked {
  uint16_t w2a[2][4][64][8];  // A operand of z2 = W2 h1: [M-tile][K-step][lane][slot]
  uint16_t w2t[2][4][64][8];  // A operand of dh1 = W2^T dz2
  float4 p1[kH];              // W1[f][0], W1[f][1], b1[f], b2[f]
  float w3[kH];
  float b3;
  float pad[3];
};

__host__ __device__ constexpr int mlp_phi(int s, int h, int i) {
  return 32 * (s >> 1) + 16 * (s & 1) + 8 * (i >> 2) + 4 * h + (i & 3);
}

struct MlpGeom {
  float f1_scale, f1_shift;  // feature 1 = ln(chi) f1_scale + f1_shift
  float f2_scale;            // feature 2 = logit(r) f2_scale
  float out_scale;           // q = out_scale y, delta = sigmoid(q + ln chi)
  float chi_lo, chi_hi;      // trained range; outside it the table samples
};

// launchers (mlp.hip)
hipError_t launch_mlp_forward(const MlpPacked* w, const float* x, float* y, int64_t n, int grid, hipStream_t st);
hipError_t launch_mlp_sample(const MlpPacked* w, MlpGeom g, TableView tab, const float* chi, const uint32_t* k,
                             float* delta, int64_t n, int grid, hipStream_t st);
// Per-wave partial gradients of the mean squared error over a batch of `batch`
// samples: sample j of the batch is data index idx(j) = base + j when seed_mode
// is 0, else floor(u n_data / 2^32) with u a Philox draw of (seed, step, j).
hipError_t launch_mlp_grad(const MlpPacked* w, const float* x, const float* t, int64_t n_data, int64_t batch,
                           int64_t base, int seed_mode, uint64_t seed, uint32_t step, float* partial,
                           hipStream_t st);
// Sums the partial rows in wave order; with adam = 0 it writes the gradient
// and the mean loss, with adam = 1 it applies one Adam step to the master
// parameters (m, v moments) and rewrites the packed forms.
struct AdamArgs {
  float lr, beta1, beta2, eps, bc1, bc2;  // bc = 1 - beta^t
};
hipError_t launch_mlp_reduce(const float* partial, int rows, int64_t batch, float* grad_out, float* loss_out,
                             float* master, float* m, float* v, MlpPacked* packed, int adam, AdamArgs a,
                             hipStream_t st);
hipError_t launch_mlp_pack(const float* master, MlpPacked* packed, hipStream_t st);

}  // namespace sfqed
