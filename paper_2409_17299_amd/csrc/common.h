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
  float s1_32;       // ln chi of the last FP32 row, s0_32 + (rows32 - 1) / inv_hs32 in FP32
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
// lo(M0 c0)); the key advances by the Weyl increments between rounds.  Each
// product is formed as one 64-bit value (one v_mad_u64_u32 on gfx950, where
// separate high and low halves take two quarter-rate multiplies).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k.y, (uint32_t)p0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ uint4 draw(uint64_t seed, uint64_t id, uint32_t step, uint32_t j) {
  return philox(make_uint4((uint32_t)id, (uint32_t)(id >> 32), step, j),
                make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
}

// -ln(u) for u = (k + 1/2) 2^-32 in FP64 (the FP64 path), and in FP32 for the
// FP32 path (event-time arithmetic is FP32; the optical depth is still
// accumulated in FP64).  For u > 1/2 the FP32 form works with v = 1 - u =
// (~k + 1/2) 2^-32, which is exact: -ln(1 - v) = -log1p(-v), evaluated with
// one logarithm as -ln(w) v / (1 - w) for w = fl(1 - v) (Goldberg, "What every
// computer scientist should know about floating-point arithmetic", 1991), or v
// when w rounds to 1.  Both halves take the same single logarithm.
__device__ __forceinline__ double exp_depth(uint32_t k) {
  return -log(((double)k + 0.5) * 0x1p-32);
}
__device__ __forceinline__ float exp_depth32(uint32_t k) {
  const bool hi = (k & 0x80000000u) != 0;
  const float v = ((float)(hi ? ~k : k) + 0.5f) * 0x1p-32f;  // u, or 1 - u
  const float w = hi ? 1.f - v : v;
  const float L = logf(w);
  if (!hi) return -L;
  return w == 1.f ? v : -L * v * __builtin_amdgcn_rcpf(1.f - w);
}
template <typename T>
__device__ __forceinline__ double exp_depth_t(uint32_t k) {
  if constexpr (sizeof(T) == 4) return (double)exp_depth32(k);
  else return exp_depth(k);
}

// ---------------------------------------------------------------------------
// Views of one species (structure of arrays) and of its fields
// (T = float or double).
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
};

template <typename T>
struct FieldView {
  const T *ex, *ey, *ez, *bx, *by, *bz;
  int64_t stride;
  int64_t n;  // entries per array when stride = 1
};

// Appended particle: one 16-byte-aligned record (the layout of qed_rec32 /
// qed_rec64), moved with whole 16-byte loads and stores.
template <typename T>
struct alignas(16) Rec {
  T px, py, pz, tb;
  double tau;
  uint64_t id;
  float w;
  uint32_t root;
  int32_t nev;
  uint32_t alive;
};
static_assert(sizeof(Rec<float>) == 48, "record layout");
static_assert(sizeof(Rec<double>) == 64, "record layout");

// A record as its 16-byte chunks, assembled and taken apart field by field (no
// type punning through memory, so the record stays in registers).
template <typename T>
struct RecBits {
  uint4 c[sizeof(Rec<T>) / 16];
};

__device__ __forceinline__ uint32_t fbits(float v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }
__device__ __forceinline__ uint64_t join64(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

template <typename T>
__device__ __forceinline__ RecBits<T> rec_pack(const Rec<T>& r) {
  RecBits<T> b;
  const uint64_t tau = __builtin_bit_cast(uint64_t, r.tau);
  const uint4 tail = make_uint4(fbits(r.w), r.root, (uint32_t)r.nev, r.alive);
  if constexpr (sizeof(T) == 4) {
    b.c[0] = make_uint4(fbits(r.px), fbits(r.py), fbits(r.pz), fbits(r.tb));
    b.c[1] = make_uint4(lo32(tau), hi32(tau), lo32(r.id), hi32(r.id));
    b.c[2] = tail;
  } else {
    const uint64_t px = __builtin_bit_cast(uint64_t, r.px), py = __builtin_bit_cast(uint64_t, r.py);
    const uint64_t pz = __builtin_bit_cast(uint64_t, r.pz), tb = __builtin_bit_cast(uint64_t, r.tb);
    b.c[0] = make_uint4(lo32(px), hi32(px), lo32(py), hi32(py));
    b.c[1] = make_uint4(lo32(pz), hi32(pz), lo32(tb), hi32(tb));
    b.c[2] = make_uint4(lo32(tau), hi32(tau), lo32(r.id), hi32(r.id));
    b.c[3] = tail;
  }
  return b;
}

template <typename T>
__device__ __forceinline__ Rec<T> rec_unpack(const RecBits<T>& b) {
  Rec<T> r;
  const uint4 tail = b.c[sizeof(T) == 4 ? 2 : 3];
  const uint4 ti = b.c[sizeof(T) == 4 ? 1 : 2];
  if constexpr (sizeof(T) == 4) {
    r.px = __builtin_bit_cast(float, b.c[0].x);
    r.py = __builtin_bit_cast(float, b.c[0].y);
    r.pz = __builtin_bit_cast(float, b.c[0].z);
    r.tb = __builtin_bit_cast(float, b.c[0].w);
  } else {
    r.px = __builtin_bit_cast(double, join64(b.c[0].x, b.c[0].y));
    r.py = __builtin_bit_cast(double, join64(b.c[0].z, b.c[0].w));
    r.pz = __builtin_bit_cast(double, join64(b.c[1].x, b.c[1].y));
    r.tb = __builtin_bit_cast(double, join64(b.c[1].z, b.c[1].w));
  }
  r.tau = __builtin_bit_cast(double, join64(ti.x, ti.y));
  r.id = join64(ti.z, ti.w);
  r.w = __builtin_bit_cast(float, tail.x);
  r.root = tail.y;
  r.nev = (int32_t)tail.z;
  r.alive = tail.w;
  return r;
}

template <typename T>
__device__ __forceinline__ void rec_load(const Rec<T>* base, int64_t i, Rec<T>& r) {
  const uint4* s = reinterpret_cast<const uint4*>(base + i);
  RecBits<T> b;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(Rec<T>) / 16); ++k) b.c[k] = s[k];
  r = rec_unpack<T>(b);
}

template <typename T>
__device__ __forceinline__ void rec_store(Rec<T>* base, int64_t i, const Rec<T>& r) {
  uint4* d = reinterpret_cast<uint4*>(base + i);
  const RecBits<T> b = rec_pack<T>(r);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(Rec<T>) / 16); ++k) d[k] = b.c[k];
}

// Stores only the 16-byte chunks [k0, k1) of a record.
template <typename T>
__device__ __forceinline__ void rec_store_part(Rec<T>* base, int64_t i, const Rec<T>& r, int k0, int k1) {
  uint4* d = reinterpret_cast<uint4*>(base + i);
  const RecBits<T> b = rec_pack<T>(r);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(Rec<T>) / 16); ++k)
    if (k >= k0 && k < k1) d[k] = b.c[k];
}

// chunk indices: momenta (and t_birth) | tau, id | w, root, nev, alive
template <typename T>
struct RecChunks {
  static constexpr int kMomEnd = sizeof(T) == 4 ? 1 : 2;
  static constexpr int kTau = kMomEnd;
  static constexpr int kTail = kMomEnd + 1;
  static constexpr int kCount = kMomEnd + 2;
};

}  // namespace sfqed
