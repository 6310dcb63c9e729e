// physics.h -- per-particle device functions of the event generator:
// chi, rates from the tables, inverse-CDF samplers, Boris push.
#pragma once

#include "common.h"

namespace sfqed {

// ---------------------------------------------------------------------------
// chi = sqrt((e E + p x B)^2 - (p.E)^2) with e = gamma for leptons and
// e = |k| for photons (the quantum parameter of a particle in E, B).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T chi_of(const T p[3], T e, const T E[3], const T B[3]) {
  const T ax = e * E[0] + (p[1] * B[2] - p[2] * B[1]);
  const T ay = e * E[1] + (p[2] * B[0] - p[0] * B[2]);
  const T az = e * E[2] + (p[0] * B[1] - p[1] * B[0]);
  const T b = p[0] * E[0] + p[1] * E[1] + p[2] * E[2];
  const T c2 = ax * ax + ay * ay + az * az - b * b;
  return c2 > T(0) ? sqrt(c2) : T(0);
}

// A photon's energy |k| and chi, and whether it can produce a pair (|k| >= 2).
// Below chi ~ 0.1 the pair rate goes as exp(-8/(3 chi)) and so multiplies a
// relative error of chi by about 8/(3 chi) (some 70 at the smallest chi whose
// rate exceeds 1e-30): the FP32 path evaluates |k| and chi from its FP32
// inputs in FP64 (full-rate enough on this chip for one evaluation per
// photon and trip) and rounds each once, which puts chi within half an ulp,
// and takes the threshold decision in FP64.  Leptons keep FP32 chi: their
// emission rate varies no faster than chi.
template <typename T>
__device__ __forceinline__ bool photon_chi(const T p[3], const T E[3], const T B[3], T& eps, T& chi) {
  if constexpr (sizeof(T) == 4) {
    const double pd[3] = {p[0], p[1], p[2]}, Ed[3] = {E[0], E[1], E[2]}, Bd[3] = {B[0], B[1], B[2]};
    const double e = sqrt(pd[0] * pd[0] + pd[1] * pd[1] + pd[2] * pd[2]);
    eps = (float)e;
    chi = (float)chi_of<double>(pd, e, Ed, Bd);
    return e >= 2.0;
  } else {
    eps = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    chi = chi_of<double>(p, eps, E, B);
    return eps >= 2.0;
  }
}

// Boris scheme over h for charge q: half electric kick, rotation in B about
// the mid-step Lorentz factor, half electric kick.
template <typename T>
__device__ __forceinline__ void boris(T p[3], T q, const T E[3], const T B[3], T h) {
  const T qh2 = T(0.5) * q * h;
  T u[3] = {p[0] + qh2 * E[0], p[1] + qh2 * E[1], p[2] + qh2 * E[2]};
  const T g = sqrt(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const T f = qh2 / g;
  const T t[3] = {f * B[0], f * B[1], f * B[2]};
  const T sc = T(2) / (T(1) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  const T v[3] = {u[0] + (u[1] * t[2] - u[2] * t[1]), u[1] + (u[2] * t[0] - u[0] * t[2]),
                  u[2] + (u[0] * t[1] - u[1] * t[0])};
  const T s[3] = {sc * t[0], sc * t[1], sc * t[2]};
  u[0] += v[1] * s[2] - v[2] * s[1];
  u[1] += v[2] * s[0] - v[0] * s[2];
  u[2] += v[0] * s[1] - v[1] * s[0];
  p[0] = u[0] + qh2 * E[0];
  p[1] = u[1] + qh2 * E[1];
  p[2] = u[2] + qh2 * E[2];
}

// ---------------------------------------------------------------------------
// Rates.  g(s), s = ln chi, is tabulated:
//   emission: g = ln(W_rad gamma / (alpha chi))
//   pairs:    g = ln(W_pair eps / (alpha chi)) + 8 / (3 chi)
// Below the table emission uses the two leading terms of the classical series
// W gamma/alpha = 5 chi/(2 sqrt3) (1 - 8 sqrt3 chi/15) and pairs are zero.
// Above it both rates approach their chi^(2/3) limits,
//   W_rad gamma / alpha -> 14 Gamma(2/3) / 3^(7/3) chi^(2/3),
//   W_pair eps / alpha  -> 15 3^(2/3) Gamma(2/3)^4 / (28 pi^2) chi^(2/3),
// as exp(a chi^(-2/3)): ln(W / chi) = ln c - s/3 + a e^(-2s/3), with a taken
// from the table's last node.
// ---------------------------------------------------------------------------
constexpr double kLnRadLimit = 0.378778931203860;    // ln(14 Gamma(2/3) / 3^(7/3))
constexpr double kLnPairLimit = -0.968604787736293;  // ln(15 3^(2/3) Gamma(2/3)^4 / (28 pi^2))

// ln(W / chi) (reduced as the table) at s > s_hi from its value l_hi at s_hi
template <typename T>
__device__ __forceinline__ T limit_continuation(T l_hi, T s_hi, T s, T ln_c) {
  return ln_c - s * T(1.0 / 3.0) + (l_hi - ln_c + s_hi * T(1.0 / 3.0)) * exp(T(-2.0 / 3.0) * (s - s_hi));
}
__device__ __forceinline__ double cheb_clenshaw(const double* c, double x) {
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int j = kChebDeg; j >= 1; --j) {
    const double b0 = fma(2.0 * x, b1, c[j] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(x, b1, 0.5 * c[0] - b2);
}

__device__ __forceinline__ double cheb_g(const RateView& r, double s) {
  const double u = (s - r.s_lo) * (1.0 / kChebSegWidth);
  int k = (int)floor(u);
  k = k < 0 ? 0 : (k >= r.nseg ? r.nseg - 1 : k);
  const double x = 2.0 * (u - k) - 1.0;
  return cheb_clenshaw(r.cheb + k * kChebN, x);
}

__device__ __forceinline__ double rate_rad64(const RateView& r, double chi, double gamma) {
  if (!(chi > 0.0)) return 0.0;
  const double s = log(chi);
  const double s_hi = r.s_lo + r.nseg * kChebSegWidth;
  double g;
  if (s < r.s_lo)
    g = log(5.0 / (2.0 * kSqrt3)) + log1p(-(8.0 * kSqrt3 / 15.0) * chi);
  else if (s > s_hi)
    g = limit_continuation<double>(cheb_g(r, s_hi), s_hi, s, kLnRadLimit);
  else
    g = cheb_g(r, s);
  return kAlpha / gamma * chi * exp(g);
}

__device__ __forceinline__ double rate_pair64(const RateView& r, double chi, double eps) {
  if (!(chi > 0.0)) return 0.0;
  const double s = log(chi);
  if (s < r.s_lo) return 0.0;
  const double s_hi = r.s_lo + r.nseg * kChebSegWidth;
  double lnf;  // ln(W eps / (alpha chi))
  if (s > s_hi) {
    const double chi_hi = exp(s_hi);
    lnf = limit_continuation<double>(cheb_g(r, s_hi) - 8.0 / (3.0 * chi_hi), s_hi, s, kLnPairLimit);
  } else {
    lnf = cheb_g(r, s) - 8.0 / (3.0 * chi);
  }
  return kAlpha / eps * chi * exp(lnf);
}

// cubic Hermite on a uniform grid (values and h-scaled slopes)
__device__ __forceinline__ float herm_g(const float2* h, int n, float t) {
  int i = (int)t;
  i = i < 0 ? 0 : (i > n - 2 ? n - 2 : i);
  const float u = t - (float)i;
  const float2 a = h[i], b = h[i + 1];
  const float u2 = u * u, u3 = u2 * u;
  const float h00 = 2.f * u3 - 3.f * u2 + 1.f, h10 = u3 - 2.f * u2 + u;
  const float h01 = -2.f * u3 + 3.f * u2, h11 = u3 - u2;
  return h00 * a.x + h10 * a.y + h01 * b.x + h11 * b.y;
}

// FP32 emission rate at chi with s = ln chi given; `herm` may point to LDS.
// The FP32 path divides through the hardware reciprocal (1 ulp).
__device__ __forceinline__ float rate_rad32_s(const float2* herm, int n, float s0, float inv_h, float chi, float s,
                                              float gamma) {
  if (!(chi > 0.f)) return 0.f;
  const float t = (s - s0) * inv_h;
  float g;
  if (t < 0.f) {
    g = 0.3669845875401003f + log1pf(-0.9237604307034012f * chi);  // ln(5/(2 sqrt3)), 8 sqrt3/15
  } else if (t > (float)(n - 1)) {
    const float th = (float)(n - 1);
    g = limit_continuation<float>(herm_g(herm, n, th), s0 + th / inv_h, s, (float)kLnRadLimit);
  } else {
    g = herm_g(herm, n, t);
  }
  return (float)kAlpha * chi * expf(g) * __builtin_amdgcn_rcpf(gamma);
}
__device__ __forceinline__ float rate_rad32(const float2* herm, int n, float s0, float inv_h, float chi,
                                            float gamma) {
  return rate_rad32_s(herm, n, s0, inv_h, chi, chi > 0.f ? logf(chi) : 0.f, gamma);
}

// FP32 pair rate (s = ln chi given).  exp(g - 8/(3 chi)) with the large
// exponent split so that its rounding does not become a relative error of the
// rate; the split is exact for any rounding of the leading quotient, because
// its residual is taken with an FMA.
__device__ __forceinline__ float rate_pair32_s(const float2* herm, int n, float s0, float inv_h, float chi, float s,
                                               float eps) {
  if (!(chi > 0.f)) return 0.f;
  const float t = (s - s0) * inv_h;
  if (t < 0.f) return 0.f;
  float g;
  if (t > (float)(n - 1)) {  // the table holds ln(W eps/(alpha chi)) + 8/(3 chi)
    const float th = (float)(n - 1);
    const float s_hi = s0 + th / inv_h;
    const float l_hi = herm_g(herm, n, th) - 2.6666667f * expf(-s_hi);
    g = limit_continuation<float>(l_hi, s_hi, s, (float)kLnPairLimit) + 2.6666667f / chi;
  } else {
    g = herm_g(herm, n, t);
  }
  const float c_hi = 2.6666667461395264f;        // 8/3 rounded to FP32
  const float c_lo = -7.947286206899662e-08f;    // 8/3 - c_hi
  const float rchi = __builtin_amdgcn_rcpf(chi);
  const float qh = c_hi * rchi;
  const float ql = (fmaf(-qh, chi, c_hi) + c_lo) * rchi;  // 8/(3 chi) = qh + ql
  const float e = g - qh;
  const float bv = e - g;
  const float err = (g - (e - bv)) + (-qh - bv);          // two-sum error of g - qh
  return (float)kAlpha * chi * expf(e) * (1.f + (err - ql)) * __builtin_amdgcn_rcpf(eps);
}
__device__ __forceinline__ float rate_pair32(const float2* herm, int n, float s0, float inv_h, float chi,
                                             float eps) {
  return rate_pair32_s(herm, n, s0, inv_h, chi, chi > 0.f ? logf(chi) : 0.f, eps);
}

// ---------------------------------------------------------------------------
// Inverse-CDF samplers.  Tables hold q on a uniform (s = ln chi, x = logit r)
// grid; 4 x 4 cubic Lagrange interpolation (stencil shifted inwards at the
// edges).  Emission: q = logit(delta) - s; below the x grid q continues as
// q(x0) + 3 (ln r - ln r0) (delta ~ r^3 for r -> 0); below the chi grid q is
// linear in chi between the first two rows (the classical limit is chi
// independent); above the chi grid chi is clamped.  Pairs: q = logit(xi) for
// r <= 1/2, mirrored for r > 1/2.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void lag4(T t, T w[4]) {
  const T tm1 = t - T(1), tm2 = t - T(2), tp1 = t + T(1);
  w[0] = -t * tm1 * tm2 * T(1.0 / 6.0);
  w[1] = tp1 * tm1 * tm2 * T(0.5);
  w[2] = -tp1 * t * tm2 * T(0.5);
  w[3] = tp1 * t * tm1 * T(1.0 / 6.0);
}

// cubic in x along one row
template <typename T, typename P>
__device__ __forceinline__ T row_interp(const P* row, int cols, T ux) {
  int j = (int)floor(ux);
  j = j < 1 ? 1 : (j > cols - 3 ? cols - 3 : j);
  T w[4];
  lag4<T>(ux - T(j), w);
  return w[0] * (T)row[j - 1] + w[1] * (T)row[j] + w[2] * (T)row[j + 1] + w[3] * (T)row[j + 2];
}

template <typename T, typename P>
__device__ __forceinline__ T grid_interp(const P* tab, int rows, int cols, T us, T ux) {
  int i = (int)floor(us);
  i = i < 1 ? 1 : (i > rows - 3 ? rows - 3 : i);
  int j = (int)floor(ux);
  j = j < 1 ? 1 : (j > cols - 3 ? cols - 3 : j);
  T ws[4], wx[4];
  lag4<T>(us - T(i), ws);
  lag4<T>(ux - T(j), wx);
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const P* r = tab + (i - 1 + a) * cols + (j - 1);
    const T v = wx[0] * (T)r[0] + wx[1] * (T)r[1] + wx[2] * (T)r[2] + wx[3] * (T)r[3];
    acc += ws[a] * v;
  }
  return acc;
}

// ln r and ln(1 - r) of r = (k + 1/2) 2^-32
__device__ __forceinline__ void log_r32(uint32_t k, float& lr, float& lrc) {
  lr = logf((float)k + 0.5f) - 22.18070977791825f;      // 32 ln 2
  lrc = logf((float)(~k) + 0.5f) - 22.18070977791825f;
}
__device__ __forceinline__ void log_r64(uint32_t k, double& lr, double& lrc) {
  lr = log((double)k + 0.5) - 32.0 * kLn2;
  lrc = log((double)(~k) + 0.5) - 32.0 * kLn2;
}
// logit r = ln((k + 1/2) / (~k + 1/2)) with one logarithm (FP32 path)
__device__ __forceinline__ float logit_r32(uint32_t k) {
  return logf(((float)k + 0.5f) * __builtin_amdgcn_rcpf((float)(~k) + 0.5f));
}
// sigmoid(z) and sigmoid(-z) from one exponential (FP32 path)
__device__ __forceinline__ void sigmoid_pair32(float z, float& p, float& q) {
  const float e = expf(-fabsf(z));
  const float r = __builtin_amdgcn_rcpf(1.f + e);
  const float small = e * r;
  p = z >= 0.f ? r : small;
  q = z >= 0.f ? small : r;
}

// Emission: z = logit(delta) at chi (s = ln chi); delta and 1 - delta are
// sigmoid(z) and sigmoid(-z).  `tab` is the FP32 grid (LDS or global).
__device__ __forceinline__ float sample_rad32_z(const float* tab, const CdfView& c, float chi, float s_chi,
                                                uint32_t k) {
  const float x = logit_r32(k);
  float ux = (x - c.x0_32) * c.inv_hx32;
  float extra = 0.f;
  if (ux < 0.f) {
    const float lr = logf((float)k + 0.5f) - 22.18070977791825f;  // ln r
    const float lr0 = -log1pf(expf(-c.x0_32));
    extra = 3.f * (lr - lr0);
    ux = 0.f;
  }
  ux = fminf(ux, (float)(c.cols32 - 1));
  const float s = fminf(s_chi, c.s1_32);  // above the grid chi is clamped
  const float us = (s - c.s0_32) * c.inv_hs32;
  float q;
  if (us < 0.f) {
    const float q0 = row_interp<float, float>(tab, c.cols32, ux);
    const float q1 = row_interp<float, float>(tab + c.cols32, c.cols32, ux);
    const float chi1 = (float)c.chi_lo * expf(1.f / c.inv_hs32);
    q = q0 + (chi - (float)c.chi_lo) / (chi1 - (float)c.chi_lo) * (q1 - q0);
  } else {
    q = grid_interp<float, float>(tab, c.rows32, c.cols32, us, ux);
  }
  return q + extra + s;
}
__device__ __forceinline__ void sample_rad32_s(const float* tab, const CdfView& c, float chi, float s_chi,
                                               uint32_t k, float& d, float& omd) {
  sigmoid_pair32(sample_rad32_z(tab, c, chi, s_chi, k), d, omd);
}
__device__ __forceinline__ void sample_rad32(const float* tab, const CdfView& c, float chi, uint32_t k, float& d,
                                             float& omd) {
  sample_rad32_s(tab, c, chi, logf(chi), k, d, omd);
}

// sigmoid(z) and sigmoid(-z) (FP64 path)
__device__ __forceinline__ void sigmoid_pair64(double z, double& p, double& q) {
  p = 1.0 / (1.0 + exp(-z));
  q = 1.0 / (1.0 + exp(z));
}

__device__ __forceinline__ double sample_rad64_z(const CdfView& c, double chi, uint32_t k) {
  double lr, lrc;
  log_r64(k, lr, lrc);
  const double x = lr - lrc;
  double ux = (x - c.x0_64) * c.inv_hx64;
  double extra = 0.0;
  if (ux < 0.0) {
    const double lr0 = -log1p(exp(-c.x0_64));
    extra = 3.0 * (lr - lr0);
    ux = 0.0;
  }
  ux = fmin(ux, (double)(c.cols64 - 1));
  const double s_max = c.s0_64 + (double)(c.rows64 - 1) / c.inv_hs64;
  const double s = fmin(log(chi), s_max);
  const double us = (s - c.s0_64) * c.inv_hs64;
  double q;
  if (us < 0.0) {
    const double q0 = row_interp<double, double>(c.f64, c.cols64, ux);
    const double q1 = row_interp<double, double>(c.f64 + c.cols64, c.cols64, ux);
    const double chi1 = c.chi_lo * exp(1.0 / c.inv_hs64);
    q = q0 + (chi - c.chi_lo) / (chi1 - c.chi_lo) * (q1 - q0);
  } else {
    q = grid_interp<double, double>(c.f64, c.rows64, c.cols64, us, ux);
  }
  return q + extra + s;
}
__device__ __forceinline__ void sample_rad64(const CdfView& c, double chi, uint32_t k, double& d, double& omd) {
  sigmoid_pair64(sample_rad64_z(c, chi, k), d, omd);
}

// Pairs: xi (electron) and 1 - xi (positron) at chi (s = ln chi).
__device__ __forceinline__ void sample_pair32_s(const float* tab, const CdfView& c, float s_chi, uint32_t k,
                                                float& xi, float& omx) {
  const float x = logit_r32(k);
  const float xa = -fabsf(x);
  float ux = fmaxf((xa - c.x0_32) * c.inv_hx32, 0.f);
  ux = fminf(ux, (float)(c.cols32 - 1));
  float us = (s_chi - c.s0_32) * c.inv_hs32;
  us = fminf(fmaxf(us, 0.f), (float)(c.rows32 - 1));
  float q = grid_interp<float, float>(tab, c.rows32, c.cols32, us, ux);
  q = fminf(q, 0.f);
  sigmoid_pair32(x > 0.f ? -q : q, xi, omx);
}
__device__ __forceinline__ void sample_pair32(const float* tab, const CdfView& c, float chi, uint32_t k, float& xi,
                                              float& omx) {
  sample_pair32_s(tab, c, logf(chi), k, xi, omx);
}

__device__ __forceinline__ void sample_pair64(const CdfView& c, double chi, uint32_t k, double& xi, double& omx) {
  double lr, lrc;
  log_r64(k, lr, lrc);
  const double x = lr - lrc;
  const double xa = -fabs(x);
  double ux = fmax((xa - c.x0_64) * c.inv_hx64, 0.0);
  ux = fmin(ux, (double)(c.cols64 - 1));
  double us = (log(chi) - c.s0_64) * c.inv_hs64;
  us = fmin(fmax(us, 0.0), (double)(c.rows64 - 1));
  double q = grid_interp<double, double>(c.f64, c.rows64, c.cols64, us, ux);
  q = fmin(q, 0.0);
  const double qq = x > 0.0 ? -q : q;
  xi = 1.0 / (1.0 + exp(-qq));
  omx = 1.0 / (1.0 + exp(qq));
}

}  // namespace sfqed
