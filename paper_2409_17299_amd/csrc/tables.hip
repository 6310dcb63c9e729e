// tables.hip -- FP64 construction of the rate and inverse-CDF tables on the GPU.
//
// Spectra (locally-constant-field nonlinear Compton and Breit-Wheeler, the
// rates the paper takes from precomputed approximations, Sec. 3):
//   emission: dW/d delta = alpha/(sqrt3 pi gamma) [A K_{2/3}(y) - Ki_{1/3}(y)],
//             A = 1 - delta + 1/(1-delta), y = 2 delta / (3 chi (1-delta));
//   pairs:    dW/d xi    = alpha/(sqrt3 pi eps)   [A K_{2/3}(y) + Ki_{1/3}(y)],
//             A = xi/(1-xi) + (1-xi)/xi,      y = 2 / (3 chi xi (1-xi));
// Ki_nu(y) = int_y^oo K_nu.
//
// Quadrature variables (both integrands are analytic and decay exponentially
// at both ends of the real line):
//   emission: w = (1/3) ln y, so z = delta/(1-delta) = 1.5 chi e^{3w} and
//             d(delta) = 4.5 chi y (1-delta)^2 dw;
//   pairs:    w = logit(xi), so y = (4/(3 chi)) (1 + cosh w) and
//             d(xi) = dw / (2 (1 + cosh w)); the integrand is even in w.
// K_{2/3} and Ki_{1/3} come from the trapezoid rule on their integral
// representations e^y K_nu(y) = int_0^oo e^{-y (cosh t - 1)} cosh(nu t) dt and
// e^y Ki_nu(y) = int_0^oo e^{-y (cosh t - 1)} cosh(nu t) / cosh t dt, which
// converges geometrically in the step for these analytic integrands.
// Integrals over w use 8-point Gauss-Legendre on panels of fixed width;
// inverse CDFs invert the cumulative panel sums by Newton iteration inside the
// panel that holds the target.

#include <algorithm>
#include <cmath>
#include <vector>

#include "lib.h"
#include "physics.h"

namespace sfqed {

constexpr double kBesselH = 0.2;  // trapezoid step in t
constexpr int kBesselN = 288;     // t up to 57.6: covers y >= 1e-20
constexpr double kYSmall = 1e-20; // below: leading small-y forms
constexpr int kGL = 8;

// emission w-panels
constexpr double kRadW0 = -40.0;
constexpr double kRadDW = 1.0 / 16.0;
constexpr int kRadPanels = 676;   // up to w = 2.25 (y = 854)
// pair half-line panels: a fixed number over [0, W(chi)], where W is the point
// beyond which the spectrum is below e^-750 of its peak
// (y - y0 = y0 sinh^2(w/2) = 750, y0 = 8/(3 chi)); the spectrum is a Gaussian
// of width ~ sqrt(2 / y0) in w at small chi, so the panels follow its width.
constexpr int kPairPanels = 152;
constexpr double kPairWMax = 19.0;

struct Consts {
  double gl_x[kGL], gl_w[kGL];        // Gauss-Legendre on [-1, 1]
  double bc[kBesselN];                // cosh(t_j) - 1
  double b23[kBesselN];               // h cosh(2 t_j / 3) (half weight at j = 0)
  double b13[kBesselN];               // h cosh(t_j / 3) / cosh(t_j)
  double k23_small, ki13_zero;        // Gamma(2/3)/2 2^{2/3}, pi/sqrt3
};

// e^{y_shift} K_{2/3}(y) and e^{y_shift} Ki_{1/3}(y), y_shift <= y (keeps the
// pair spectrum in range far below its threshold).  The trapezoid rule in t
// loses accuracy like exp(-2 pi^2 / (h^2 y)) as y grows, because the integrand
// narrows to a Gaussian of width 1/sqrt(y); above y = 4 the substitution
// y (cosh t - 1) = v^2, t = 2 asinh(v / sqrt(2y)), dt = 2 dv / sqrt(2y + v^2)
// turns it into e^{-v^2} times a function analytic in |Im v| < sqrt(2y), and
// the trapezoid rule in v converges like exp(-pi^2 / h^2).
constexpr double kBesselHv = 0.25;
constexpr int kBesselNv = 27;  // v up to 6.5

__device__ void bessel_pair(const Consts& c, double y, double y_shift, double& k23, double& ki13) {
  if (y - y_shift > 745.0) {
    k23 = 0.0;
    ki13 = 0.0;
    return;
  }
  const double e = exp(-(y - y_shift));
  if (y < kYSmall) {
    k23 = e * c.k23_small * pow(y, -2.0 / 3.0);
    ki13 = e * c.ki13_zero;
    return;
  }
  double s23 = 0.0, s13 = 0.0;
  if (y > 4.0) {
    const double r2y = 1.0 / sqrt(2.0 * y), iy = 1.0 / y;
    for (int j = kBesselNv - 1; j >= 0; --j) {
      const double v = j * kBesselHv;
      const double a = asinh(v * r2y);
      const double wv = (j == 0 ? 0.5 : 1.0) * kBesselHv * exp(-v * v) * 2.0 * r2y / sqrt(1.0 + v * v * r2y * r2y);
      const double c23 = cosh(a * (4.0 / 3.0)), c13 = cosh(a * (2.0 / 3.0));
      s23 = fma(wv, c23, s23);
      s13 = fma(wv, c13 / (1.0 + v * v * iy), s13);
    }
  } else {
    // terms with y (cosh t - 1) > 745 underflow
    int jmax = (int)(acosh(1.0 + 745.0 / y) * (1.0 / kBesselH)) + 1;
    jmax = jmax < kBesselN - 1 ? jmax : kBesselN - 1;
    for (int j = jmax; j >= 0; --j) {  // small terms first
      const double a = y * c.bc[j];
      if (a > 745.0) continue;
      const double ej = exp(-a);
      s23 = fma(c.b23[j], ej, s23);
      s13 = fma(c.b13[j], ej, s13);
    }
  }
  k23 = s23 * e;
  ki13 = s13 * e;
}

// emission integrand in w (reduced by alpha/gamma)
__device__ double rad_integrand(const Consts& c, double chi, double w) {
  const double y = exp(3.0 * w);
  const double z = 1.5 * chi * y;
  const double omd = 1.0 / (1.0 + z);
  const double a = omd + (1.0 + z);
  double k23, ki13;
  bessel_pair(c, y, 0.0, k23, ki13);
  return (a * k23 - ki13) * (1.0 / (kSqrt3 * kPi)) * 4.5 * chi * y * omd * omd;
}

// pair integrand in w (reduced by alpha/eps), scaled by e^{8/(3 chi)}
__device__ double pair_integrand(const Consts& c, double chi, double w) {
  const double ch = cosh(w);
  const double y0 = 8.0 / (3.0 * chi);
  const double sh = sinh(0.5 * w);
  const double y = y0 + y0 * sh * sh;  // (4/(3chi))(1 + cosh w) = y0 cosh^2(w/2)
  double k23, ki13;
  bessel_pair(c, y, y0, k23, ki13);
  return (2.0 * ch * k23 + ki13) * (1.0 / (kSqrt3 * kPi)) / (2.0 * (1.0 + ch));
}

template <int P>
__device__ double integrand(const Consts& c, double chi, double w) {
  return P == 0 ? rad_integrand(c, chi, w) : pair_integrand(c, chi, w);
}

template <int P>
__device__ double gl_panel(const Consts& c, double chi, double a, double b) {
  const double m = 0.5 * (a + b), h = 0.5 * (b - a);
  double s = 0.0;
  for (int i = 0; i < kGL; ++i) s = fma(c.gl_w[i], integrand<P>(c, chi, fma(h, c.gl_x[i], m)), s);
  return s * h;
}

// panel k spans [g.w0 + k g.dw, g.w0 + (k+1) g.dw]
struct Panels {
  double w0, dw;
};

template <int P>
__device__ __forceinline__ Panels panels_for(double chi) {
  if (P == 0) return Panels{kRadW0, kRadDW};
  const double y0 = 8.0 / (3.0 * chi);
  const double W = fmin(kPairWMax, 2.0 * asinh(sqrt(750.0 / y0)));
  return Panels{0.0, W / kPairPanels};
}
template <int P>
__device__ __forceinline__ int npanels() {
  return P == 0 ? kRadPanels : kPairPanels;
}

// Deterministic block sum in FP64 (fixed tree order).
__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Reduced rate integral at chi: emission: int over the whole w line;
// pairs: twice the half line (scaled by e^{8/(3chi)}).
template <int P>
__device__ double reduced_total(const Consts& c, double chi, double* red) {
  const Panels pg = panels_for<P>(chi);
  double acc = 0.0;
  for (int k = threadIdx.x; k < npanels<P>(); k += blockDim.x)
    acc += gl_panel<P>(c, chi, pg.w0 + k * pg.dw, pg.w0 + (k + 1) * pg.dw);
  double tot = block_sum(acc, red);
  if (P == 0) tot += integrand<0>(c, chi, kRadW0);  // tail below w0 ~ e^w
  else tot *= 2.0;
  return tot;
}

__global__ void __launch_bounds__(256) k_rate_nodes(const Consts* cg, int process, double s_lo, double* g_out) {
  __shared__ Consts c;
  __shared__ double red[256];
  for (int i = threadIdx.x; i < (int)(sizeof(Consts) / sizeof(double)); i += blockDim.x)
    reinterpret_cast<double*>(&c)[i] = reinterpret_cast<const double*>(cg)[i];
  __syncthreads();
  const int seg = blockIdx.x / kChebN, m = blockIdx.x % kChebN;
  const double xm = cos(kPi * (m + 0.5) / kChebN);
  const double s = s_lo + seg * kChebSegWidth + 0.5 * kChebSegWidth * (xm + 1.0);
  const double chi = exp(s);
  double tot;
  if (process == 0)
    tot = reduced_total<0>(c, chi, red);
  else
    tot = reduced_total<1>(c, chi, red);
  if (threadIdx.x == 0) g_out[blockIdx.x] = log(tot) - s;  // pairs: + 8/(3chi) is in the scaling
}

// c_j = (2/N) sum_m g_m cos(j pi (m + 1/2) / N)
__global__ void k_cheb_coeffs(const double* g, int nseg, double* coef) {
  const int seg = blockIdx.x, j = threadIdx.x;
  if (seg >= nseg || j >= kChebN) return;
  double acc = 0.0;
  for (int m = 0; m < kChebN; ++m) acc += g[seg * kChebN + m] * cos(kPi * j * (m + 0.5) / kChebN);
  coef[seg * kChebN + j] = 2.0 * acc / kChebN;
}

// FP32 Hermite nodes: g and h g' from the Chebyshev series.
__global__ void k_rate_herm(const double* coef, int nseg, double s_lo, int n, double h, float2* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = s_lo + i * h;
  double u = (s - s_lo) / kChebSegWidth;
  int k = (int)floor(u);
  k = k < 0 ? 0 : (k >= nseg ? nseg - 1 : k);
  const double x = 2.0 * (u - k) - 1.0;
  const double* c = coef + k * kChebN;
  const double g = cheb_clenshaw(c, x);
  // derivative series: d_{j-1} = d_{j+1} + 2 j c_j
  double d[kChebN + 1];
  d[kChebN] = 0.0;
  d[kChebN - 1] = 0.0;
  for (int j = kChebN - 1; j >= 1; --j) d[j - 1] = (j + 1 <= kChebN ? d[j + 1] : 0.0) + 2.0 * j * c[j];
  const double dg_dx = cheb_clenshaw(d, x);  // uses d[0..16]
  const double dg_ds = dg_dx * (2.0 / kChebSegWidth);
  out[i] = make_float2((float)g, (float)(h * dg_ds));
}

// One row of an inverse-CDF grid: chi = exp(s0 + row hs); columns x0 + j hx.
template <int P>
__global__ void __launch_bounds__(256) k_cdf_rows(const Consts* cg, double s0, double hs, double x0, double hx,
                                                  int cols, float* out32, double* out64) {
  __shared__ Consts c;
  __shared__ double I[kRadPanels];
  __shared__ double C[kRadPanels + 1], D[kRadPanels + 1];
  for (int i = threadIdx.x; i < (int)(sizeof(Consts) / sizeof(double)); i += blockDim.x)
    reinterpret_cast<double*>(&c)[i] = reinterpret_cast<const double*>(cg)[i];
  __syncthreads();
  const int row = blockIdx.x;
  const double s = s0 + row * hs;
  const double chi = exp(s);
  const int np = npanels<P>();
  const Panels pg = panels_for<P>(chi);
  for (int k = threadIdx.x; k < np; k += blockDim.x) I[k] = gl_panel<P>(c, chi, pg.w0 + k * pg.dw, pg.w0 + (k + 1) * pg.dw);
  __syncthreads();
  if (threadIdx.x == 0) {
    C[0] = P == 0 ? integrand<0>(c, chi, kRadW0) : 0.0;
    for (int k = 0; k < np; ++k) C[k + 1] = C[k] + I[k];
    D[np] = 0.0;
    for (int k = np - 1; k >= 0; --k) D[k] = D[k + 1] + I[k];
  }
  __syncthreads();
  const double total = P == 0 ? C[np] : 2.0 * D[0];
  for (int j = threadIdx.x; j < cols; j += blockDim.x) {
    const double x = x0 + j * hx;
    const double r = 1.0 / (1.0 + exp(-x)), rc = 1.0 / (1.0 + exp(x));
    // find the panel and the integral still to cover inside it, from its left edge
    int k;
    double loc;
    if (P == 0 && x <= 0.0) {
      const double T = r * total;
      int lo = 0, hi = np;  // C[lo] <= T < C[hi]
      if (T < C[0]) { lo = 0; hi = 0; }
      while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (C[mid] <= T) lo = mid; else hi = mid;
      }
      k = lo;
      loc = T - C[k];
    } else {
      // from the top: find k with D[k+1] <= T < D[k]
      const double T = P == 0 ? rc * total : r * total;  // pairs: half line from the top = r * total
      int lo = 0, hi = np;  // D[lo] > T >= D[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (D[mid] > T) lo = mid; else hi = mid;
      }
      k = lo;
      loc = I[k] - (T - D[k + 1]);
    }
    k = k < 0 ? 0 : (k >= np ? np - 1 : k);
    const double a = pg.w0 + k * pg.dw, b = a + pg.dw;
    double wlo = a, whi = b;
    double w = a + (b - a) * fmin(1.0, fmax(0.0, I[k] > 0.0 ? loc / I[k] : 0.5));
    for (int it = 0; it < 60; ++it) {
      const double G = gl_panel<P>(c, chi, a, w) - loc;
      if (G > 0.0) whi = w; else wlo = w;
      const double f = integrand<P>(c, chi, w);
      double wn = f > 0.0 ? w - G / f : 0.5 * (wlo + whi);
      if (!(wn > wlo && wn < whi)) wn = 0.5 * (wlo + whi);
      const bool done = fabs(wn - w) <= 1e-15 * fmax(1.0, fabs(w)) || whi - wlo <= 1e-15 * fmax(1.0, fabs(w));
      w = wn;
      if (done) break;
    }
    double q;
    if (P == 0) q = log(1.5) + 3.0 * w;  // logit(delta) - ln chi
    else q = -w;                         // logit(xi) for xi <= 1/2
    if (out32) out32[row * cols + j] = (float)q;
    if (out64) out64[row * cols + j] = q;
  }
}

// ------------------------------------------------------------------ host side
namespace {

void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      dp = n * (z * p1 - p2) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // recompute the derivative at the converged node
        double q1 = 1.0, q2 = 0.0;
        for (int j = 1; j <= n; ++j) {
          const double q3 = q2;
          q2 = q1;
          q1 = ((2.0 * j - 1.0) * z * q2 - (j - 1.0) * q3) / j;
        }
        dp = n * (z * q1 - q2) / (z * z - 1.0);
        break;
      }
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

qed_status build_tables(const qed_table_cfg& cfg, hipStream_t stream, qed_tables* t) {
  TableGeom& g = t->geom;
  g.cfg = cfg;
  // Chebyshev rate ranges: emission from rate_chi_min, pairs from max(rate_chi_min, 1e-3)
  const double lo[2] = {std::log(cfg.rate_chi_min), std::log(std::max(cfg.rate_chi_min, 1e-3))};
  const double hi = std::log(cfg.rate_chi_max);
  for (int p = 0; p < 2; ++p) {
    g.cheb_s_lo[p] = lo[p];
    g.nseg[p] = (int)std::ceil((hi - lo[p]) / kChebSegWidth);
  }
  g.herm_n = cfg.rate_nodes;
  g.rows32[0] = cfg.rad_rows;
  g.cols32[0] = cfg.rad_cols;
  g.rows32[1] = cfg.pair_rows;
  g.cols32[1] = cfg.pair_cols;
  for (int p = 0; p < 2; ++p) {
    g.rows64[p] = (g.rows32[p] - 1) * cfg.f64_refine + 1;
    g.cols64[p] = (g.cols32[p] - 1) * cfg.f64_refine + 1;
  }
  g.s0[0] = std::log(cfg.rad_chi_min);
  g.s1[0] = std::log(cfg.rad_chi_max);
  g.x0[0] = cfg.rad_x_min;
  g.x1[0] = cfg.rad_x_max;
  g.s0[1] = std::log(cfg.pair_chi_min);
  g.s1[1] = std::log(cfg.pair_chi_max);
  g.x0[1] = cfg.pair_x_min;
  g.x1[1] = 0.0;

  // layout of the single allocation
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t o_consts = take(sizeof(Consts));
  size_t o_nodes[2], o_cheb[2], o_herm[2], o_c32[2], o_c64[2];
  for (int p = 0; p < 2; ++p) {
    o_nodes[p] = take(sizeof(double) * g.nseg[p] * kChebN);
    o_cheb[p] = take(sizeof(double) * g.nseg[p] * kChebN);
    o_herm[p] = take(sizeof(float2) * g.herm_n);
    o_c32[p] = take(sizeof(float) * g.rows32[p] * g.cols32[p]);
    o_c64[p] = take(sizeof(double) * g.rows64[p] * g.cols64[p]);
  }
  t->bytes = off;
  SFQED_HIP(hipMalloc(&t->mem, t->bytes));
  char* base = static_cast<char*>(t->mem);

  Consts hc;
  gauss_legendre(kGL, hc.gl_x, hc.gl_w);
  for (int j = 0; j < kBesselN; ++j) {
    const double tj = j * kBesselH;
    const double sh = std::sinh(0.5 * tj);
    hc.bc[j] = 2.0 * sh * sh;
    const double wj = (j == 0 ? 0.5 : 1.0) * kBesselH;
    hc.b23[j] = wj * std::cosh(2.0 * tj / 3.0);
    hc.b13[j] = wj * std::cosh(tj / 3.0) / std::cosh(tj);
  }
  hc.k23_small = 0.5 * std::tgamma(2.0 / 3.0) * std::pow(2.0, 2.0 / 3.0);
  hc.ki13_zero = kPi / kSqrt3;
  Consts* dconsts = reinterpret_cast<Consts*>(base + o_consts);
  SFQED_HIP(hipMemcpyAsync(dconsts, &hc, sizeof(Consts), hipMemcpyHostToDevice, stream));

  for (int p = 0; p < 2; ++p) {
    double* nodes = reinterpret_cast<double*>(base + o_nodes[p]);
    double* cheb = reinterpret_cast<double*>(base + o_cheb[p]);
    float2* herm = reinterpret_cast<float2*>(base + o_herm[p]);
    hipLaunchKernelGGL(k_rate_nodes, dim3(g.nseg[p] * kChebN), dim3(256), 0, stream, dconsts, p, g.cheb_s_lo[p],
                       nodes);
    hipLaunchKernelGGL(k_cheb_coeffs, dim3(g.nseg[p]), dim3(32), 0, stream, nodes, g.nseg[p], cheb);
    const double hs = g.nseg[p] * kChebSegWidth / (g.herm_n - 1);
    hipLaunchKernelGGL(k_rate_herm, dim3((g.herm_n + 255) / 256), dim3(256), 0, stream, cheb, g.nseg[p],
                       g.cheb_s_lo[p], g.herm_n, hs, herm);
    RateView& rv = t->view.rate[p];
    rv.cheb = cheb;
    rv.s_lo = g.cheb_s_lo[p];
    rv.nseg = g.nseg[p];
    rv.herm = herm;
    rv.hs_lo = (float)g.cheb_s_lo[p];
    rv.inv_h = (float)(1.0 / hs);
    rv.n = g.herm_n;

    float* c32 = reinterpret_cast<float*>(base + o_c32[p]);
    double* c64 = reinterpret_cast<double*>(base + o_c64[p]);
    const double hs32 = (g.s1[p] - g.s0[p]) / (g.rows32[p] - 1), hx32 = (g.x1[p] - g.x0[p]) / (g.cols32[p] - 1);
    const double hs64 = (g.s1[p] - g.s0[p]) / (g.rows64[p] - 1), hx64 = (g.x1[p] - g.x0[p]) / (g.cols64[p] - 1);
    if (p == 0) {
      hipLaunchKernelGGL(k_cdf_rows<0>, dim3(g.rows32[p]), dim3(256), 0, stream, dconsts, g.s0[p], hs32, g.x0[p],
                         hx32, g.cols32[p], c32, (double*)nullptr);
      hipLaunchKernelGGL(k_cdf_rows<0>, dim3(g.rows64[p]), dim3(256), 0, stream, dconsts, g.s0[p], hs64, g.x0[p],
                         hx64, g.cols64[p], (float*)nullptr, c64);
    } else {
      hipLaunchKernelGGL(k_cdf_rows<1>, dim3(g.rows32[p]), dim3(256), 0, stream, dconsts, g.s0[p], hs32, g.x0[p],
                         hx32, g.cols32[p], c32, (double*)nullptr);
      hipLaunchKernelGGL(k_cdf_rows<1>, dim3(g.rows64[p]), dim3(256), 0, stream, dconsts, g.s0[p], hs64, g.x0[p],
                         hx64, g.cols64[p], (float*)nullptr, c64);
    }
    SFQED_HIP(hipGetLastError());
    CdfView& cv = t->view.cdf[p];
    cv.f32 = c32;
    cv.rows32 = g.rows32[p];
    cv.cols32 = g.cols32[p];
    cv.s0_32 = (float)g.s0[p];
    cv.inv_hs32 = (float)(1.0 / hs32);
    cv.x0_32 = (float)g.x0[p];
    cv.inv_hx32 = (float)(1.0 / hx32);
    cv.s1_32 = cv.s0_32 + (float)(cv.rows32 - 1) / cv.inv_hs32;
    cv.f64 = c64;
    cv.rows64 = g.rows64[p];
    cv.cols64 = g.cols64[p];
    cv.s0_64 = g.s0[p];
    cv.inv_hs64 = 1.0 / hs64;
    cv.x0_64 = g.x0[p];
    cv.inv_hx64 = 1.0 / hx64;
    cv.chi_lo = std::exp(g.s0[p]);
    cv.chi_hi = std::exp(g.s1[p]);

    t->off[0 + p] = o_cheb[p];
    t->len[0 + p] = sizeof(double) * g.nseg[p] * kChebN;
    t->off[2 + p] = o_herm[p];
    t->len[2 + p] = sizeof(float2) * g.herm_n;
    t->off[4 + p] = o_c32[p];
    t->len[4 + p] = sizeof(float) * g.rows32[p] * g.cols32[p];
    t->off[6 + p] = o_c64[p];
    t->len[6 + p] = sizeof(double) * g.rows64[p] * g.cols64[p];
  }
  return QED_OK;
}

}  // namespace sfqed
