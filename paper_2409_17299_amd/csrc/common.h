// common.h -- device-side definitions shared by the kernels of libsfqed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfqed {

// fine-structure constant (CODATA 2018)
constexpr double kAlpha = 7.2973525693e-3;
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kSqrt3 = 1.73205080756887729352744634150587237;
constexpr double kLn2 = 0.693147180559945309417232121458176568;

constexpr int kChebDeg = 16;          // FP64 rate: Chebyshev degree per segment
constexpr int kChebN = kChebDeg + 1;  // coefficients per segment
constexpr double kChebSegWidth = 0.5; // in ln chi

// ---------------------------------------------------------------------------
// Table views passed to kernels by value.
// ---------------------------------------------------------------------------
struct RateView {
  const double* cheb;  // [nseg][kChebN]; g(s) on [s_lo, s_lo + nseg/2]
  double s_lo;
  int nseg;
  const float2* herm;  // [n]: g(s_i), h g'(s_i); s_i = hs_lo + i h
  float hs_lo, inv_h;
  int n;
};

struct CdfView {
  const float* f32;  // [rows32][cols32]
  int rows32, cols32;
  float s0_32, inv_hs32, x0_32, inv_hx32;
  const double* f64;  // [rows64][cols64]
  int rows64, cols64;
  double s0_64, inv_hs64, x0_64, inv_hx64;
  double chi_lo, chi_hi;  // chi of the first and last row
};

struct TableView {
  RateView rate[2];  // 0 emission, 1 pairs
  CdfView cdf[2];
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One round maps
// (c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)); the key advances by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ uint4 draw(uint64_t seed, uint64_t id, uint32_t step, uint32_t j) {
  return philox(make_uint4((uint32_t)id, (uint32_t)(id >> 32), step, j),
                make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
}

// -ln(u) for u = (k + 1/2) 2^-32, in FP64 (optical depths are FP64)
__device__ __forceinline__ double exp_depth(uint32_t k) {
  return -log(((double)k + 0.5) * 0x1p-32);
}

// ---------------------------------------------------------------------------
// Views of one species and of its fields (T = float or double).
// ---------------------------------------------------------------------------
template <typename T>
struct SpeciesView {
  T *px, *py, *pz;
  T *x, *y, *z;  // nullable
  float* w;
  double* tau;
  uint64_t* id;
  uint8_t* alive;  // nullable for leptons
  int32_t* nev;    // nullable
  uint32_t* root;  // nullable: then root = species << 30 | index
  T* tb;           // nullable: then 0
};

template <typename T>
struct FieldView {
  const T *ex, *ey, *ez, *bx, *by, *bz;
  int64_t stride;
};

}  // namespace sfqed
