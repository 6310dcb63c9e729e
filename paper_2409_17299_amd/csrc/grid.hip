// grid.hip -- the field stage in front of the QED step: given fields on a
// periodic line of nodes along x (the plane-wave test problem of Sec. 5.1),
// periodic wrapping of particle positions and linear interpolation of the
// fields at them into per-particle arrays, plus the standing circularly
// polarised wave of that test problem as a field source.
//
// Both kernels are bound by HBM: the gather reads a particle's position and
// writes its six field components (36 bytes per particle in FP32, 72 in
// FP64; a position is written back only when the wrap moves it).  A grid of
// up to kGatherLdsNodes nodes is copied into each block's LDS first, so the
// interpolation reads it at LDS latency.  Arithmetic is FP64 in a fixed order with no
// fused operations, so the stored values are a function of the inputs alone.

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "lib.h"

#pragma clang fp contract(off)

namespace sfqed {
namespace {

constexpr int kGatherThreads = 256;
constexpr int kGatherItems = 4;
constexpr int kGatherTile = kGatherThreads * kGatherItems;
constexpr int kGatherLdsNodes = 1024;  // grids up to this size are staged in LDS (24 KB FP32, 48 KB FP64)

template <typename T>
struct GatherSpecies {
  T* pos[3];
  T* out[6];
  int64_t n;
  int64_t first_block;  // blocks [first_block, first_block + ceil(n / tile)) cover this species
};

template <typename T>
struct GatherArgs {
  GatherSpecies<T> s[3];
  const T* g[6];
  double nxd, x0, rdx;         // nodes (as a double), first node, nx / length
  double lo[3], len[3], rlen[3], hi[3];
  int32_t wrap[3];
};

// x' = x - floor((x - lo) / len) len, kept inside [lo, lo + len) against the
// rounding of the reciprocal and of the product.
__device__ __forceinline__ double wrap_coord(double x, double lo, double len, double rlen, double hi) {
  const double s = floor((x - lo) * rlen);
  double w = x - s * len;
  if (w < lo)
    w = w + len;
  else if (w >= hi)
    w = w - len;
  return w;
}

// One particle: wrap its coordinates (v, as loaded), store those that moved,
// and write the grid's field at its stored x.  g: the six node arrays (LDS or
// global).
template <typename T>
__device__ __forceinline__ void gather_one(const GatherArgs<T>& a, const GatherSpecies<T>& S, const T* const* g,
                                           int64_t i, const T (&v)[3]) {
  double xs = 0.0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    T t = v[ax];
    if (a.wrap[ax]) {
      t = (T)wrap_coord((double)v[ax], a.lo[ax], a.len[ax], a.rlen[ax], a.hi[ax]);
      if (t != v[ax]) S.pos[ax][i] = t;
    }
    if (ax == 0) xs = (double)t;
  }
  const double u = (xs - a.x0) * a.rdx;
  const double q = floor(u);
  const double f = u - q;
  double ic = q - a.nxd * floor(q / a.nxd);
  ic = fmin(fmax(ic, 0.0), a.nxd - 1.0);  // NaN goes to node 0
  const int i0 = (int)ic;
  const int i1 = (double)(i0 + 1) == a.nxd ? 0 : i0 + 1;
  const double h = 1.0 - f;
#pragma unroll
  for (int c = 0; c < 6; ++c) S.out[c][i] = (T)(h * (double)g[c][i0] + f * (double)g[c][i1]);
}

// Blocks are laid out species by species, kGatherTile particles each; a full
// tile issues all its position loads before any arithmetic.  Grids of up to
// kGatherLdsNodes nodes are first copied to LDS.
template <typename T>
__global__ __launch_bounds__(kGatherThreads) void k_gather(GatherArgs<T> a) {
  extern __shared__ __align__(16) unsigned char gather_lds[];  // 6 nx values when nx <= kGatherLdsNodes
  T* const lds = reinterpret_cast<T*>(gather_lds);
  const int64_t b = blockIdx.x;
  const int sp = b >= a.s[2].first_block ? 2 : (b >= a.s[1].first_block ? 1 : 0);
  const GatherSpecies<T>& S = a.s[sp];
  const int nx = (int)a.nxd;
  const T* g[6];
  if (nx <= kGatherLdsNodes) {
    for (int k = threadIdx.x; k < 6 * nx; k += kGatherThreads) lds[k] = a.g[k / nx][k % nx];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 6; ++c) g[c] = lds + c * nx;
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) g[c] = a.g[c];
  }
  const int64_t tile = (b - S.first_block) * kGatherTile;
  if (tile + kGatherTile <= S.n) {
    T v[kGatherItems][3];
#pragma unroll
    for (int it = 0; it < kGatherItems; ++it)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) v[it][ax] = S.pos[ax][tile + threadIdx.x + it * kGatherThreads];
#pragma unroll
    for (int it = 0; it < kGatherItems; ++it) gather_one(a, S, g, tile + threadIdx.x + it * kGatherThreads, v[it]);
  } else {
    for (int it = 0; it < kGatherItems; ++it) {
      const int64_t i = tile + threadIdx.x + it * kGatherThreads;
      if (i >= S.n) break;
      const T v[3] = {S.pos[0][i], S.pos[1][i], S.pos[2][i]};
      gather_one(a, S, g, i, v);
    }
  }
}

template <typename T>
struct WaveArgs {
  T* g[6];
  int64_t nx;
  double x0, dx, xc, k, e0, ct, st;
};

template <typename T>
__global__ __launch_bounds__(256) void k_standing_wave(WaveArgs<T> a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nx) return;
  const double x = a.x0 + (double)i * a.dx;
  const double phi = a.k * (x - a.xc);
  const double ce = a.e0 * cos(phi);
  const double sb = a.e0 * sin(phi);
  a.g[0][i] = (T)0.0;
  a.g[1][i] = (T)(ce * a.ct);
  a.g[2][i] = (T)(ce * a.st);
  a.g[3][i] = (T)0.0;
  a.g[4][i] = (T)(sb * a.ct);
  a.g[5][i] = (T)(sb * a.st);
}

bool grid_ok(const qed_grid1d& g) {
  if (g.nx < 1 || !std::isfinite(g.x0) || !std::isfinite(g.length) || !(g.length > 0.0)) return false;
  if (g.dtype != QED_F32 && g.dtype != QED_F64) return false;
  return g.ex && g.ey && g.ez && g.bx && g.by && g.bz;
}

template <typename T>
qed_status gather_impl(qed_ensemble* ens, const qed_grid1d& g, const qed_box& box, const qed_field_arrays* out,
                       hipStream_t st) {
  GatherArgs<T> a{};
  int64_t blocks = 0;
  for (int s = 0; s < 3; ++s) {
    const qed_species& sp = ens->s[s];
    GatherSpecies<T>& S = a.s[s];
    S.pos[0] = static_cast<T*>(sp.x);
    S.pos[1] = static_cast<T*>(sp.y);
    S.pos[2] = static_cast<T*>(sp.z);
    void* const o[6] = {out[s].ex, out[s].ey, out[s].ez, out[s].bx, out[s].by, out[s].bz};
    for (int c = 0; c < 6; ++c) S.out[c] = static_cast<T*>(o[c]);
    S.n = sp.count;
    S.first_block = blocks;
    blocks += (sp.count + kGatherTile - 1) / kGatherTile;
  }
  const void* const gv[6] = {g.ex, g.ey, g.ez, g.bx, g.by, g.bz};
  for (int c = 0; c < 6; ++c) a.g[c] = static_cast<const T*>(gv[c]);
  if (g.nx > 0x7FFFFFFF) {
    set_error("gather_fields: too many nodes");
    return QED_ERR_ARG;
  }
  a.nxd = (double)g.nx;
  a.x0 = g.x0;
  a.rdx = (double)g.nx / g.length;
  for (int ax = 0; ax < 3; ++ax) {
    a.wrap[ax] = box.len[ax] > 0.0;
    a.lo[ax] = box.lo[ax];
    a.len[ax] = box.len[ax];
    a.rlen[ax] = a.wrap[ax] ? 1.0 / box.len[ax] : 0.0;
    a.hi[ax] = box.lo[ax] + box.len[ax];
  }
  if (blocks == 0) return QED_OK;
  if (blocks > 0x7FFFFFFF) {
    set_error("gather_fields: too many particles for one launch");
    return QED_ERR_ARG;
  }
  const size_t lds = g.nx <= kGatherLdsNodes ? 6 * (size_t)g.nx * sizeof(T) : 0;
  hipLaunchKernelGGL((k_gather<T>), dim3((unsigned)blocks), dim3(kGatherThreads), lds, st, a);
  SFQED_HIP(hipGetLastError());
  return QED_OK;
}

template <typename T>
qed_status wave_impl(const qed_grid1d& g, double e0, double k, double omega, double xc, double t, hipStream_t st) {
  WaveArgs<T> a{};
  void* const gv[6] = {g.ex, g.ey, g.ez, g.bx, g.by, g.bz};
  for (int c = 0; c < 6; ++c) a.g[c] = static_cast<T*>(gv[c]);
  a.nx = g.nx;
  a.x0 = g.x0;
  a.dx = g.length / (double)g.nx;
  a.xc = xc;
  a.k = k;
  a.e0 = e0;
  a.ct = std::cos(omega * t);
  a.st = std::sin(omega * t);
  const int64_t blocks = (g.nx + 255) / 256;
  if (blocks > 0x7FFFFFFF) {
    set_error("grid_standing_wave: too many nodes");
    return QED_ERR_ARG;
  }
  hipLaunchKernelGGL((k_standing_wave<T>), dim3((unsigned)blocks), dim3(256), 0, st, a);
  SFQED_HIP(hipGetLastError());
  return QED_OK;
}

}  // namespace
}  // namespace sfqed

using sfqed::set_error;

extern "C" {

qed_status qed_grid_standing_wave(const qed_grid1d* g, double e0, double k, double omega, double xc, double t,
                                  void* stream) {
  if (!g || !sfqed::grid_ok(*g) || !std::isfinite(e0) || !std::isfinite(k) || !std::isfinite(omega) ||
      !std::isfinite(xc) || !std::isfinite(t)) {
    set_error("grid_standing_wave: invalid grid or wave parameters");
    return QED_ERR_ARG;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  return g->dtype == QED_F32 ? sfqed::wave_impl<float>(*g, e0, k, omega, xc, t, st)
                             : sfqed::wave_impl<double>(*g, e0, k, omega, xc, t, st);
}

qed_status qed_gather_fields(qed_ensemble* ens, const qed_grid1d* g, const qed_box* box,
                             const qed_field_arrays out[3], void* stream) {
  if (!ens || !g || !box || !out) return QED_ERR_ARG;
  if (!sfqed::grid_ok(*g) || g->dtype != ens->dtype) {
    set_error("gather_fields: invalid grid, or its dtype differs from the ensemble's");
    return QED_ERR_ARG;
  }
  for (int ax = 0; ax < 3; ++ax) {
    if (!std::isfinite(box->lo[ax]) || !std::isfinite(box->len[ax]) || box->len[ax] < 0.0) {
      set_error("gather_fields: invalid box");
      return QED_ERR_ARG;
    }
  }
  for (int s = 0; s < 3; ++s) {
    const qed_species& sp = ens->s[s];
    if (sp.count < 0 || sp.count > sp.capacity) {
      set_error("gather_fields: invalid count of species " + std::to_string(s));
      return QED_ERR_ARG;
    }
    if (sp.count == 0) continue;
    const qed_field_arrays& o = out[s];
    if (!sp.x || !sp.y || !sp.z || !o.ex || !o.ey || !o.ez || !o.bx || !o.by || !o.bz) {
      set_error("gather_fields: species " + std::to_string(s) + " needs positions and six output arrays");
      return QED_ERR_ARG;
    }
    if (o.n < sp.count) {
      set_error("gather_fields: the output arrays of species " + std::to_string(s) + " hold fewer entries than " +
                std::to_string(sp.count) + " particles");
      return QED_ERR_ARG;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ens->dtype == QED_F32) return sfqed::gather_impl<float>(ens, *g, *box, out, st);
  if (ens->dtype == QED_F64) return sfqed::gather_impl<double>(ens, *g, *box, out, st);
  return QED_ERR_ARG;
}

}  // extern "C"
