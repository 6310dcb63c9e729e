// mlp.hip -- inference and training kernels of the inverse-CDF surrogate
// (2 -> 64 -> 64 -> 1, SiLU).  One wave evaluates 32 samples at a time: lane l
// and lane l + 32 share sample l % 32 and each holds 32 of the 64 hidden
// features of every layer (the slot mapping of mlp.h).  Layer 2 and the
// back-propagation through it are BF16 MFMA with FP32 accumulation (BF16
// weights; activations as a hi + lo pair of bfloat16 numbers); the weight
// gradients are MFMA products over the sample dimension after an LDS
// transpose.  Reductions over waves are in a fixed order, so a training run is
// deterministic.
#include "mlp.h"
#include "physics.h"

namespace sfqed {

namespace {

__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

__device__ __forceinline__ bf16x8 frag_load(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

// The parameters one lane needs, in registers for the whole kernel.
struct LaneParams {
  bf16x8 w2[2][4];
  float4 p1[32];  // slot s*8+i: W1[phi][0], W1[phi][1], b1[phi], b2[phi]
  float w3[32];
  float b3;
};

__device__ __forceinline__ void load_params(const MlpPacked* W, int lane, LaneParams& P) {
  const int h = lane >> 5;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int s = 0; s < 4; ++s) P.w2[mt][s] = frag_load(W->w2a[mt][s][lane]);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int f = mlp_phi(s, h, i);
      P.p1[s * 8 + i] = W->p1[f];
      P.w3[s * 8 + i] = W->w3[f];
    }
  P.b3 = W->b3;
}

// Layer 1 in FP32 and its SiLU.  Each activation leaves as two bfloat16
// numbers, hi = bf16(h) and lo = bf16(h - hi), the B operands of layer 2, so
// that the product sees h to about 16 significant bits (z1 and sigmoid(z1)
// optionally kept for the backward pass).
template <bool kKeep>
__device__ __forceinline__ void layer1(const LaneParams& P, float f1, float f2, bf16x8 hb[4], bf16x8 lb[4],
                                       float* z1, float* s1) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float4 q = P.p1[s * 8 + i];
      const float z = fmaf(q.x, f1, fmaf(q.y, f2, q.z));
      const float sg = sigm(z);
      const float h = z * sg;
      const __bf16 hi = (__bf16)h;
      hb[s][i] = hi;
      lb[s][i] = (__bf16)(h - (float)hi);
      if constexpr (kKeep) {
        z1[s * 8 + i] = z;
        s1[s * 8 + i] = sg;
      }
    }
}

// z2 (without bias) = W2 (hi + lo), or W2 b for a single operand.
__device__ __forceinline__ void layer2(const bf16x8 w[2][4], const bf16x8 b[4], const bf16x8* lo, f32x16 acc[2]) {
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 c = {};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      c = mfma(w[mt][s], b[s], c);
      if (lo) c = mfma(w[mt][s], lo[s], c);
    }
    acc[mt] = c;
  }
}

// Network output for the lane's sample (both lanes of a sample get it).
__device__ __forceinline__ float forward(const LaneParams& P, float f1, float f2) {
  bf16x8 hb[4], lb[4];
  layer1<false>(P, f1, f2, hb, lb, nullptr, nullptr);
  f32x16 acc[2];
  layer2(P.w2, hb, lb, acc);
  float y = 0.f;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float z = acc[mt][r] + P.p1[16 * mt + r].w;
      y = fmaf(P.w3[16 * mt + r], z * sigm(z), y);
    }
  y += __shfl_xor(y, 32);
  return y + P.b3;
}

// Inference keeps the W2 fragments and the layer-1 weights in registers and
// reads the biases and w3 (per feature slot) from LDS, where the two halves of
// a wave each read one address: 96 fewer registers per lane, two waves per
// SIMD instead of one.
struct InferParams {
  bf16x8 w2[2][4];
  float w1a[32], w1b[32];  // slot s*8+i: feature phi(s, h, i)
  float b3;
};

// For h = 0, 1 and slot = 0..31 (feature f = phi(slot / 8, h, slot % 8)):
// l1[h][slot] = b1[f], l3[h][slot] = (b2[f], w3[f]).  The whole block calls
// this (it synchronises).
__device__ __forceinline__ void load_infer_params(const MlpPacked* W, int lane, InferParams& P, float (*l1)[32],
                                                  float2 (*l3)[32]) {
  const int h = lane >> 5;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int s = 0; s < 4; ++s) P.w2[mt][s] = frag_load(W->w2a[mt][s][lane]);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float4 q = W->p1[mlp_phi(s, h, i)];
      P.w1a[s * 8 + i] = q.x;
      P.w1b[s * 8 + i] = q.y;
    }
  P.b3 = W->b3;
  if (threadIdx.x < 64) {
    const int hh = threadIdx.x >> 5, q = threadIdx.x & 31, f = mlp_phi(q >> 3, hh, q & 7);
    l1[hh][q] = W->p1[f].z;
    l3[hh][q] = make_float2(W->p1[f].w, W->w3[f]);
  }
  __syncthreads();
}

__device__ __forceinline__ float forward_infer(const InferParams& P, const float* l1h, const float2* l3h, float f1,
                                               float f2) {
  // layer 1 one K-step at a time, each step's activations going straight into
  // its four MFMAs (fewer values live at once)
  f32x16 acc[2] = {f32x16{}, f32x16{}};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    bf16x8 hb, lb;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int q = s * 8 + i;
      const float z = fmaf(P.w1a[q], f1, fmaf(P.w1b[q], f2, l1h[q]));
      const float h = z * sigm(z);
      const __bf16 hi = (__bf16)h;
      hb[i] = hi;
      lb[i] = (__bf16)(h - (float)hi);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      acc[mt] = mfma(P.w2[mt][s], hb, acc[mt]);
      acc[mt] = mfma(P.w2[mt][s], lb, acc[mt]);
    }
  }
  float y = 0.f;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float2 c = l3h[16 * mt + r];
      const float z = acc[mt][r] + c.x;
      y = fmaf(c.y, z * sigm(z), y);
    }
  y += __shfl_xor(y, 32);
  return y + P.b3;
}

__global__ void __launch_bounds__(kMlpThreads, 2) k_mlp_forward(const MlpPacked* W, const float* x, float* y,
                                                                int64_t n) {
  __shared__ float l1[2][32];
  __shared__ float2 l3[2][32];
  const int lane = threadIdx.x & 63;
  InferParams P;
  load_infer_params(W, lane, P, l1, l3);
  const float* l1h = l1[lane >> 5];
  const float2* l3h = l3[lane >> 5];
  const int64_t nw = (int64_t)gridDim.x * (kMlpThreads / 64);
  for (int64_t t = (int64_t)blockIdx.x * (kMlpThreads / 64) + (threadIdx.x >> 6); t * 32 < n; t += nw) {
    const int64_t i = t * 32 + (lane & 31);
    const bool ok = i < n;
    const float f1 = ok ? x[2 * i] : 0.f, f2 = ok ? x[2 * i + 1] : 0.f;
    const float v = forward_infer(P, l1h, l3h, f1, f2);
    if (ok && lane < 32) y[i] = v;
  }
}

// delta = sigmoid(out_scale y + ln chi) inside the trained chi range, the FP32
// table sampler outside it.
__global__ void __launch_bounds__(kMlpThreads, 2) k_mlp_sample(const MlpPacked* W, MlpGeom g, TableView tab,
                                                              const float* chi, const uint32_t* k, float* delta,
                                                              int64_t n) {
  __shared__ float l1[2][32];
  __shared__ float2 l3[2][32];
  const int lane = threadIdx.x & 63;
  InferParams P;
  load_infer_params(W, lane, P, l1, l3);
  const float* l1h = l1[lane >> 5];
  const float2* l3h = l3[lane >> 5];
  const int64_t nw = (int64_t)gridDim.x * (kMlpThreads / 64);
  for (int64_t t = (int64_t)blockIdx.x * (kMlpThreads / 64) + (threadIdx.x >> 6); t * 32 < n; t += nw) {
    const int64_t i = t * 32 + (lane & 31);
    const bool ok = i < n;
    const float c = ok ? chi[i] : 1.f;
    const uint32_t kk = ok ? k[i] : 0x80000000u;
    float lr, lrc;
    log_r32(kk, lr, lrc);
    const float lc = logf(c);
    const float v = forward_infer(P, l1h, l3h, fmaf(lc, g.f1_scale, g.f1_shift), (lr - lrc) * g.f2_scale);
    float d = sigm(fmaf(v, g.out_scale, lc));
    if (!(c >= g.chi_lo && c <= g.chi_hi)) {
      float omd;
      sample_rad32(tab.cdf[0].f32, tab.cdf[0], c, kk, d, omd);
    }
    if (ok && lane < 32) delta[i] = d;
  }
}

// ------------------------------------------------------------------ training
constexpr int kGradThreads = 128;  // two waves, one 32-sample tile each
constexpr int kRows = 260;         // LDS rows per wave: dz2, dz1, h2, h1 (64 each), f1, f2, 1, dy
constexpr int kRowDz2 = 0, kRowDz1 = 64, kRowH2 = 128, kRowH1 = 192, kRowX = 256;

__device__ __forceinline__ uint32_t batch_index(int64_t j, int64_t n_data, int64_t base, int seed_mode,
                                                uint64_t seed, uint32_t step) {
  if (seed_mode) {
    const uint4 u = draw(seed, (uint64_t)j, step, 0x4D4C5000u);
    return (uint32_t)(((uint64_t)u.x * (uint64_t)n_data) >> 32);
  }
  int64_t i = base + j;
  if (i >= n_data) i -= n_data;
  return (uint32_t)i;
}

__global__ void __launch_bounds__(kGradThreads) k_mlp_grad(const MlpPacked* W, const float* x, const float* t,
                                                          int64_t n_data, int64_t batch, int64_t base, int seed_mode,
                                                          uint64_t seed, uint32_t step, float* partial) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[kGradThreads / 64][kRows][32];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
  const int64_t tile = (int64_t)blockIdx.x * (kGradThreads / 64) + wv;
  LaneParams P;
  load_params(W, lane, P);
  bf16x8 w2t[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int s = 0; s < 4; ++s) w2t[mt][s] = frag_load(W->w2t[mt][s][lane]);

  const int64_t j = tile * 32 + col;
  const bool ok = j < batch;
  float f1 = 0.f, f2 = 0.f, tt = 0.f;
  if (ok) {
    const uint32_t i = batch_index(j, n_data, base, seed_mode, seed, step);
    f1 = x[2 * (int64_t)i];
    f2 = x[2 * (int64_t)i + 1];
    tt = t[i];
  }
  // forward, keeping what the backward pass needs
  bf16x8 hb[4], lb[4];
  float z1[32], s1[32];
  layer1<true>(P, f1, f2, hb, lb, z1, s1);
  f32x16 acc[2];
  layer2(P.w2, hb, lb, acc);
  float z2[32], s2[32], y = 0.f;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int q = 16 * mt + r;
      z2[q] = acc[mt][r] + P.p1[q].w;
      s2[q] = sigm(z2[q]);
      y = fmaf(P.w3[q], z2[q] * s2[q], y);
    }
  y += __shfl_xor(y, 32);
  y += P.b3;
  const float res = ok ? y - tt : 0.f;
  const float dy = res * (2.f / (float)batch);

  // dz2 = dy w3 silu'(z2) -> B operands of dh1 = W2^T dz2
  bf16x8 db[4];
  float dz2[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    dz2[q] = dy * P.w3[q] * s2[q] * fmaf(z2[q], 1.f - s2[q], 1.f);
    db[q >> 3][q & 7] = (__bf16)dz2[q];
  }
  f32x16 dacc[2];
  layer2(w2t, db, nullptr, dacc);

  // transpose through LDS: row = feature (or input), column = sample
  uint16_t(*L)[32] = lds[wv];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int q = s * 8 + i, f = mlp_phi(s, h, i);
      const float dz1 = dacc[q >> 4][q & 15] * s1[q] * fmaf(z1[q], 1.f - s1[q], 1.f);
      L[kRowDz2 + f][col] = bf16_bits(dz2[q]);
      L[kRowDz1 + f][col] = bf16_bits(dz1);
      L[kRowH2 + f][col] = bf16_bits(z2[q] * s2[q]);
      // the leading bfloat16 part of h1, from the same FP32 value the forward
      // rounded (elements are not read back out of the bf16 vectors)
      L[kRowH1 + f][col] = bf16_bits(z1[q] * s1[q]);
    }
  if (h == 0) {
    L[kRowX + 0][col] = bf16_bits(f1);
    L[kRowX + 1][col] = bf16_bits(f2);
    L[kRowX + 2][col] = bf16_bits(ok ? 1.f : 0.f);
    L[kRowX + 3][col] = bf16_bits(dy);
  }
  __syncthreads();

  // weight gradients: sums over the tile's 32 samples (two K-steps of 16)
  f32x16 gw2[2][2], ge[6];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) gw2[a][b] = f32x16{};
#pragma unroll
  for (int a = 0; a < 6; ++a) ge[a] = f32x16{};
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int c0 = 16 * kk + 8 * h;
    bf16x8 bh[2], bx;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) bh[nt] = frag_load(&L[kRowH1 + 32 * nt + col][c0]);
    bx = col < 4 ? frag_load(&L[kRowX + col][c0]) : bf16x8{};
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const bf16x8 af = frag_load(&L[32 * a + col][c0]);
      if (a < 2) {
        gw2[a][0] = mfma(af, bh[0], gw2[a][0]);
        gw2[a][1] = mfma(af, bh[1], gw2[a][1]);
      }
      ge[a] = mfma(af, bx, ge[a]);
    }
  }

  // per-wave partial row
  float* out = partial + tile * kGradRow;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r >> 2) + 4 * h + (r & 3);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) out[kOffW2 + kH * (32 * a + row) + 32 * b + col] = gw2[a][b][r];
    if (col == 2) {
      out[kOffB2 + row] = ge[0][r];
      out[kOffB2 + 32 + row] = ge[1][r];
      out[kOffB1 + row] = ge[2][r];
      out[kOffB1 + 32 + row] = ge[3][r];
    } else if (col < 2) {
      out[kOffW1 + 2 * row + col] = ge[2][r];
      out[kOffW1 + 2 * (32 + row) + col] = ge[3][r];
    } else if (col == 3) {
      out[kOffW3 + row] = ge[4][r];
      out[kOffW3 + 32 + row] = ge[5][r];
    }
  }
  // b3 and the squared residuals: sums over the 32 samples, fixed order
  float gb = h == 0 ? dy : 0.f, sq = h == 0 ? res * res : 0.f;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    gb += __shfl_xor(gb, o);
    sq += __shfl_xor(sq, o);
  }
  if (lane == 0) {
    out[kOffB3] = gb;
    out[kMlpParams] = sq;
  }
}

// Writes parameter i of the master copy into the packed forms.
__device__ __forceinline__ void pack_one(MlpPacked* P, int i, float v) {
  if (i < kOffB1) {
    float* p = reinterpret_cast<float*>(&P->p1[i >> 1]);
    p[i & 1] = v;
  } else if (i < kOffW2) {
    P->p1[i - kOffB1].z = v;
  } else if (i < kOffB2) {
    const int f = (i - kOffW2) >> 6, k = (i - kOffW2) & 63;
    const uint16_t b = bf16_bits(v);
    // z2 = W2 h1: row f, K index k
    {
      const int s = 2 * (k >> 5) + ((k >> 4) & 1), hh = (k >> 2) & 1, sl = 4 * ((k >> 3) & 1) + (k & 3);
      P->w2a[f >> 5][s][(f & 31) + 32 * hh][sl] = b;
    }
    // dh1 = W2^T dz2: row k, K index f
    {
      const int s = 2 * (f >> 5) + ((f >> 4) & 1), hh = (f >> 2) & 1, sl = 4 * ((f >> 3) & 1) + (f & 3);
      P->w2t[k >> 5][s][(k & 31) + 32 * hh][sl] = b;
    }
  } else if (i < kOffW3) {
    P->p1[i - kOffB2].w = v;
  } else if (i < kOffB3) {
    P->w3[i - kOffW3] = v;
  } else {
    P->b3 = v;
  }
}

__global__ void k_mlp_pack(const float* master, MlpPacked* P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) pack_one(P, i, master[i]);
}

__global__ void k_mlp_reduce(const float* partial, int rows, int64_t batch, float* grad_out, float* loss_out,
                             float* master, float* m, float* v, MlpPacked* P, int adam, AdamArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kGradRow) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += (double)partial[(int64_t)r * kGradRow + i];
  if (i == kMlpParams) {
    if (loss_out) *loss_out = (float)(s / (double)batch);
    return;
  }
  const float g = (float)s;
  if (!adam) {
    grad_out[i] = g;
    return;
  }
  const float mi = a.beta1 * m[i] + (1.f - a.beta1) * g;
  const float vi = a.beta2 * v[i] + (1.f - a.beta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float p = master[i] - a.lr * (mi / a.bc1) / (sqrtf(vi / a.bc2) + a.eps);
  master[i] = p;
  pack_one(P, i, p);
}

}  // namespace

hipError_t launch_mlp_forward(const MlpPacked* w, const float* x, float* y, int64_t n, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(kMlpThreads), 0, st, w, x, y, n);
  return hipGetLastError();
}

hipError_t launch_mlp_sample(const MlpPacked* w, MlpGeom g, TableView tab, const float* chi, const uint32_t* k,
                             float* delta, int64_t n, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_sample, dim3(grid), dim3(kMlpThreads), 0, st, w, g, tab, chi, k, delta, n);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpPacked* w, const float* x, const float* t, int64_t n_data, int64_t batch,
                           int64_t base, int seed_mode, uint64_t seed, uint32_t step, float* partial,
                           hipStream_t st) {
  const int64_t blocks = (batch + kGradThreads / 2 - 1) / (kGradThreads / 2);
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)blocks), dim3(kGradThreads), 0, st, w, x, t, n_data, batch, base,
                     seed_mode, seed, step, partial);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float* partial, int rows, int64_t batch, float* grad_out, float* loss_out,
                             float* master, float* m, float* v, MlpPacked* packed, int adam, AdamArgs a,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kGradRow + 255) / 256), dim3(256), 0, st, partial, rows, batch, grad_out,
                     loss_out, master, m, v, packed, adam, a);
  return hipGetLastError();
}

hipError_t launch_mlp_pack(const float* master, MlpPacked* packed, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, master, packed);
  return hipGetLastError();
}

}  // namespace sfqed
