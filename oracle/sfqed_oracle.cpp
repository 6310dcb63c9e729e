// sfqed_oracle.cpp -- TEST INFRASTRUCTURE, not part of the product.
//
// A plain, slow, FP64 CPU reference for the per-macroparticle strong-field QED
// event generator of arXiv:2409.17299 (inverse sampling with sub-cycling,
// Sec. 3, Algorithms 1 and 2).  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg load this library.  It shares no source with the
// HIP library: its special functions, quadrature, random-number generator and
// sampler are written here from their definitions.
//
// Units: momenta in m_e c, electric fields in E_S = m_e^2 c^3/(e hbar), magnetic
// fields in E_S/c, times in hbar/(m_e c^2), lengths in hbar/(m_e c).  With these
// units dp/dt = q (E + p x B / gamma) and the quantum parameter is
// chi = |F_{mu nu} p^nu| / (m c E_S).
//
// Physics the paper names but does not write down (Sec. 3 defers the rates to
// polynomial fits of the "first and second synchrotron functions"): the
// locally-constant-field nonlinear Compton and Breit-Wheeler spectra,
//
//   dW_rad/d delta = alpha/(sqrt3 pi gamma) [ (1-d+1/(1-d)) K_{2/3}(y) - Ki_{1/3}(y) ],
//                    y = 2 d / (3 chi (1-d)),  d = photon energy / lepton energy,
//   dW_pair/d xi   = alpha/(sqrt3 pi eps)   [ (xi/(1-xi)+(1-xi)/xi) K_{2/3}(y) + Ki_{1/3}(y) ],
//                    y = 2 / (3 chi xi (1-xi)),  xi = electron energy / photon energy,
//
// with K_nu the modified Bessel function of the second kind and
// Ki_nu(y) = int_y^inf K_nu(s) ds.
//
// Two tiers:
//  * definitions tier: K_nu and Ki_nu by adaptive Gauss-Legendre quadrature of
//    their integral representations (DLMF 10.32.9), used for pins and to check
//    the fast tier;
//  * ensemble tier: the same spectra with K_{2/3} and Ki_{1/3} read from a fine
//    table of the definitions tier (10-point Lagrange in ln y), so that a whole
//    ensemble step runs in seconds.  Rates are integrals of the spectrum and
//    samples are exact inversions of its cumulative integral (no rate or
//    inverse-CDF table), so the method's own approximations are not repeated.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

namespace {

constexpr double kAlpha = 7.2973525693e-3;   // fine-structure constant (CODATA 2018)
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kSqrt3 = 1.73205080756887729352744634150587237;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (c0,c1,c2,c3) -> (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0)),
// with the key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// Stream layout: key = seed, counter = (id_lo, id_hi, step, j).
void draw(uint64_t seed, uint64_t id, uint32_t step, uint32_t j, uint32_t out[4]) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, j};
  philox4x32_10(ctr, key, out);
}

// Uniform on (0,1): r = (k + 1/2) 2^-32, exact in FP64, never 0 or 1.  The
// complement 1 - r = (~k + 1/2) 2^-32 is exact as well.
inline double u01(uint32_t k) { return ((double)k + 0.5) * 0x1p-32; }
inline double u01c(uint32_t k) { return ((double)(~k) + 0.5) * 0x1p-32; }

// ---------------------------------------------------------------------------
// Adaptive Gauss-Legendre quadrature.  The n-point rule's nodes are found by
// Newton iteration on the Legendre polynomial P_n (three-term recurrence).  A
// panel's error is |G(panel) - G(left half) - G(right half)|; the panel with the
// largest error is split until the summed error meets the tolerance.
// ---------------------------------------------------------------------------
struct GaussLegendre {
  static constexpr int N = 20;
  double x[N], w[N];
  GaussLegendre() {
    for (int i = 0; i < N; ++i) {
      double z = std::cos(kPi * (i + 0.75) / (N + 0.5));
      double dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= N; ++j) {
          const double p3 = p2;
          p2 = p1;
          p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        dp = N * (z * p1 - p2) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-17) break;
      }
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= N; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      dp = N * (z * p1 - p2) / (z * z - 1.0);
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};
const GaussLegendre& gl() {
  static const GaussLegendre rule;
  return rule;
}

template <class F>
double gl_panel(const F& f, double a, double b) {
  const GaussLegendre& r = gl();
  const double c = 0.5 * (a + b), h = 0.5 * (b - a);
  double s = 0.0;
  for (int i = 0; i < GaussLegendre::N; ++i) s += r.w[i] * f(c + h * r.x[i]);
  return s * h;
}

struct Panel {
  double a, b, whole, left, right;
  double val() const { return left + right; }
  double err() const { return std::fabs(whole - left - right); }
};

// Integrates f over the consecutive intervals given by `breaks` (sorted).
// Returns the accepted panels in order of position.
template <class F>
std::vector<Panel> quad_panels(const F& f, const std::vector<double>& breaks, double rtol,
                               double atol, int max_panels = 3000) {
  std::vector<Panel> ps;
  ps.reserve(breaks.size() * 4);
  auto make = [&](double a, double b, double whole) {
    const double m = 0.5 * (a + b);
    Panel p{a, b, whole, gl_panel(f, a, m), gl_panel(f, m, b)};
    return p;
  };
  for (size_t i = 0; i + 1 < breaks.size(); ++i) {
    const double a = breaks[i], b = breaks[i + 1];
    if (!(b > a)) continue;
    ps.push_back(make(a, b, gl_panel(f, a, b)));
  }
  while ((int)ps.size() < max_panels) {
    double tot = 0.0, err = 0.0;
    size_t worst = 0;
    double werr = -1.0;
    for (size_t i = 0; i < ps.size(); ++i) {
      tot += ps[i].val();
      const double e = ps[i].err();
      err += e;
      if (e > werr) { werr = e; worst = i; }
    }
    if (err <= std::max(atol, rtol * std::fabs(tot))) break;
    const Panel p = ps[worst];
    const double m = 0.5 * (p.a + p.b);
    if (!(m > p.a && m < p.b)) break;
    ps[worst] = make(p.a, m, p.left);
    ps.insert(ps.begin() + worst + 1, make(m, p.b, p.right));
  }
  return ps;
}

template <class F>
double quad(const F& f, const std::vector<double>& breaks, double rtol, double atol = 0.0) {
  const std::vector<Panel> ps = quad_panels(f, breaks, rtol, atol);
  double s = 0.0;
  for (const Panel& p : ps) s += p.val();
  return s;
}

// ---------------------------------------------------------------------------
// Definitions tier of the special functions (DLMF 10.32.9 and its integral):
//   e^x K_nu(x)              = int_0^inf exp(-x (cosh t - 1)) cosh(nu t)          dt
//   e^x int_x^inf K_nu(s) ds = int_0^inf exp(-x (cosh t - 1)) cosh(nu t) / cosh t dt
// The upper limit T is where the integrand has fallen below e^-70 of its size
// near the origin.
// ---------------------------------------------------------------------------
double cutoff_t(double nu, double x) {
  double T = std::acosh(1.0 + 70.0 / x);
  for (int it = 0; it < 8; ++it) T = std::acosh(1.0 + (70.0 + nu * T) / x);
  return T;
}

std::vector<double> t_breaks(double nu, double x) {
  const double T = cutoff_t(nu, x);
  std::vector<double> br{0.0};
  // the integrand turns over near t ~ ln(2 nu / x) for small x
  for (double t = 0.5; t < T; t *= 2.0) br.push_back(t);
  br.push_back(T);
  return br;
}

double bessel_k_scaled_def(double nu, double x) {
  auto f = [&](double t) {
    const double sh = std::sinh(0.5 * t);
    return std::exp(-x * 2.0 * sh * sh) * std::cosh(nu * t);
  };
  return quad(f, t_breaks(nu, x), 1e-15);
}

double bessel_ki_scaled_def(double nu, double x) {
  auto f = [&](double t) {
    const double sh = std::sinh(0.5 * t);
    return std::exp(-x * 2.0 * sh * sh) * std::cosh(nu * t) / std::cosh(t);
  };
  return quad(f, t_breaks(nu, x), 1e-15);
}

// ---------------------------------------------------------------------------
// Fast tier: ln(e^y K_{2/3}(y)) and ln(e^y Ki_{1/3}(y)) tabulated against
// s = ln y on a uniform grid, read back by 10-point Lagrange interpolation.
// Below the grid the y -> 0 limits K_{2/3} = Gamma(2/3)/2 (2/y)^{2/3} and
// Ki_{1/3} = pi/sqrt3 hold to far better than FP64 (corrections are O(y^{2/3})
// with y < 1e-45); above it, e^-y underflows.
// ---------------------------------------------------------------------------
constexpr double kSLo = -104.0;           // ln(1e-45) ~ -103.6
constexpr double kSHi = 6.625;            // ln(750) ~ 6.62
constexpr double kSH = 0.025;
constexpr int kNS = (int)((kSHi - kSLo) / kSH + 0.5) + 1;
constexpr int kLag = 10;

struct SpecialTables {
  std::vector<double> lk23, lki13;
  SpecialTables() : lk23(kNS), lki13(kNS) {
    for (int i = 0; i < kNS; ++i) {
      const double y = std::exp(kSLo + kSH * i);
      lk23[i] = std::log(bessel_k_scaled_def(2.0 / 3.0, y));
      lki13[i] = std::log(bessel_ki_scaled_def(1.0 / 3.0, y));
    }
  }
};

const SpecialTables& special_tables() {
  static const SpecialTables t;  // thread-safe static initialisation
  return t;
}

// Lagrange weights of the kLag nodes i0 .. i0+kLag-1 at grid coordinate u,
// l_i(u) = prod_{j != i} (u - j) / prod_{j != i} (i - j).
struct LagrangeWeights {
  int i0;
  double l[kLag];
  explicit LagrangeWeights(double s) {
    const double u = (s - kSLo) / kSH;
    i0 = (int)std::floor(u) - (kLag / 2 - 1);
    i0 = std::max(0, std::min(kNS - kLag, i0));
    static const std::vector<double> inv_den = [] {
      std::vector<double> d(kLag);
      for (int i = 0; i < kLag; ++i) {
        double p = 1.0;
        for (int j = 0; j < kLag; ++j)
          if (j != i) p *= (double)(i - j);
        d[i] = 1.0 / p;
      }
      return d;
    }();
    double pre[kLag + 1], suf[kLag + 1];
    pre[0] = 1.0;
    for (int j = 0; j < kLag; ++j) pre[j + 1] = pre[j] * (u - (i0 + j));
    suf[kLag] = 1.0;
    for (int j = kLag - 1; j >= 0; --j) suf[j] = suf[j + 1] * (u - (i0 + j));
    for (int i = 0; i < kLag; ++i) l[i] = pre[i] * suf[i + 1] * inv_den[i];
  }
  double apply(const std::vector<double>& v) const {
    double acc = 0.0;
    for (int i = 0; i < kLag; ++i) acc += l[i] * v[i0 + i];
    return acc;
  }
};

const double kGamma23 = std::tgamma(2.0 / 3.0);

// Both functions at one y (they share the grid, so the weights are shared).
void k23_ki13_fast(double y, double* k, double* ki) {
  if (y > 745.0) {
    *k = 0.0;
    *ki = 0.0;
    return;
  }
  const double s = std::log(y);
  if (s < kSLo) {
    *k = 0.5 * kGamma23 * std::pow(2.0 / y, 2.0 / 3.0);
    *ki = kPi / kSqrt3;
    return;
  }
  const SpecialTables& t = special_tables();
  const LagrangeWeights lw(s);
  *k = std::exp(lw.apply(t.lk23) - y);
  *ki = std::exp(lw.apply(t.lki13) - y);
}

void k23_ki13(double y, bool def, double* k, double* ki) {
  if (def) {
    *k = std::exp(-y) * bessel_k_scaled_def(2.0 / 3.0, y);
    *ki = std::exp(-y) * bessel_ki_scaled_def(1.0 / 3.0, y);
  } else {
    k23_ki13_fast(y, k, ki);
  }
}

double k23(double y, bool def) {
  double k, ki;
  if (def) return std::exp(-y) * bessel_k_scaled_def(2.0 / 3.0, y);
  k23_ki13_fast(y, &k, &ki);
  return k;
}

double ki13(double y, bool def) {
  double k, ki;
  if (def) return std::exp(-y) * bessel_ki_scaled_def(1.0 / 3.0, y);
  k23_ki13_fast(y, &k, &ki);
  return ki;
}

// ---------------------------------------------------------------------------
// Spectra, reduced by the prefactor alpha/gamma (alpha/eps for pairs), so that
// W_rad = alpha/gamma * int_0^1 spec_rad d(delta) and likewise for pairs.
// ---------------------------------------------------------------------------
double spec_rad(double chi, double d, double omd, bool def) {
  // d = delta, omd = 1 - delta (passed separately to keep it exact near 1)
  if (!(d > 0.0) || !(omd > 0.0)) return 0.0;
  const double y = 2.0 * d / (3.0 * chi * omd);
  const double a = omd + 1.0 / omd;
  double k, ki;
  k23_ki13(y, def, &k, &ki);
  return (a * k - ki) / (kSqrt3 * kPi);
}

double spec_pair(double chi, double xi, double omx, bool def) {
  if (!(xi > 0.0) || !(omx > 0.0)) return 0.0;
  const double y = 2.0 / (3.0 * chi * xi * omx);
  const double a = xi / omx + omx / xi;
  double k, ki;
  k23_ki13(y, def, &k, &ki);
  return (a * k + ki) / (kSqrt3 * kPi);
}

// Emission is integrated in v, y = v^3, with z = delta/(1-delta) = 3 chi y / 2:
//   d(delta) = dz/(1+z)^2, dz = (3 chi / 2) 3 v^2 dv.
// The v^2 Jacobian cancels the y^{-2/3} end-point singularity and the spectrum
// falls off as exp(-v^3), so the integrand is smooth on [0, 9.1].
struct RadVar {
  double chi;
  bool def;
  double operator()(double v) const {
    const double y = v * v * v;
    const double z = 1.5 * chi * y;
    const double d = z / (1.0 + z), omd = 1.0 / (1.0 + z);
    return spec_rad(chi, d, omd, def) * omd * omd * 1.5 * chi * 3.0 * v * v;
  }
};
constexpr double kVMax = 9.1;  // y = 753: e^-y underflows beyond

std::vector<double> rad_breaks(double chi) {
  // the Jacobian varies on the scale z ~ 1, i.e. v ~ (2/(3 chi))^{1/3}
  const double vc = std::cbrt(2.0 / (3.0 * chi));
  std::vector<double> br{0.0};
  for (double f : {1.0 / 16, 1.0 / 8, 1.0 / 4, 1.0 / 2, 1.0, 2.0, 4.0}) {
    const double v = f * vc;
    if (v < kVMax) br.push_back(v);
  }
  for (double v : {0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0}) br.push_back(v);
  br.push_back(kVMax);
  std::sort(br.begin(), br.end());
  br.erase(std::unique(br.begin(), br.end()), br.end());
  return br;
}

// Pairs are integrated over xi in (0, 1/2] and doubled (the spectrum is
// symmetric under xi <-> 1-xi).  Features sit near xi ~ 1/chi (large chi) and
// within ~ sqrt(chi)/4 of xi = 1/2 (small chi).
struct PairVar {
  double chi;
  bool def;
  double operator()(double xi) const { return spec_pair(chi, xi, 1.0 - xi, def); }
};

std::vector<double> pair_breaks(double chi) {
  std::vector<double> br{0.0, 0.5};
  const double xc = 1.0 / (3.0 * chi);
  for (double f = 1.0 / 64; f <= 64.0; f *= 2.0)
    if (f * xc < 0.5) br.push_back(f * xc);
  const double wc = 0.25 * std::sqrt(chi);
  for (double f = 1.0 / 4; f <= 16.0; f *= 2.0)
    if (f * wc < 0.5) br.push_back(0.5 - f * wc);
  std::sort(br.begin(), br.end());
  br.erase(std::unique(br.begin(), br.end()), br.end());
  return br;
}

constexpr double kRtol = 1e-14;

double rate_rad_reduced(double chi, bool def) {
  if (!(chi > 0.0)) return 0.0;
  return quad(RadVar{chi, def}, rad_breaks(chi), kRtol);
}

double rate_pair_reduced(double chi, bool def) {
  if (!(chi > 0.0)) return 0.0;
  return 2.0 * quad(PairVar{chi, def}, pair_breaks(chi), kRtol);
}

// Solves int_{a}^{x} f = target inside one accepted panel [a, b] by safeguarded
// Newton iteration (f is the density, so the derivative is exact).
template <class F>
double invert_in_panel(const F& f, double a, double b, double target, double panel_val) {
  double lo = a, hi = b;
  double x = a + (b - a) * std::min(1.0, std::max(0.0, target / panel_val));
  for (int it = 0; it < 100; ++it) {
    const double g = gl_panel(f, a, x) - target;
    if (g > 0.0) hi = x; else lo = x;
    const double d = f(x);
    double xn = (d > 0.0) ? x - g / d : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (std::fabs(xn - x) <= 1e-16 * std::fabs(x) || hi - lo <= 1e-16 * std::fabs(x)) {
      x = xn;
      break;
    }
    x = xn;
  }
  return x;
}

// The accepted panels of one spectrum with their running sums from the bottom
// (lo[k] = panels 0..k) and from the top (hi[k] = panels k..end), accumulated in
// the order a sequential scan would use.
struct CdfPanels {
  std::vector<Panel> ps;
  std::vector<double> lo, hi;
  double tot = 0.0;
};

template <class F>
CdfPanels cdf_panels(const F& f, const std::vector<double>& breaks) {
  CdfPanels c;
  c.ps = quad_panels(f, breaks, kRtol, 0.0);
  const size_t n = c.ps.size();
  c.lo.resize(n);
  c.hi.resize(n);
  double cum = 0.0;
  for (size_t k = 0; k < n; ++k) c.lo[k] = cum += c.ps[k].val();
  c.tot = cum;
  cum = 0.0;
  for (size_t k = n; k-- > 0;) c.hi[k] = cum += c.ps[k].val();
  return c;
}

// Returns x with int_0^x f = r * total, using the complement from the top end
// when r > 1/2 (rc = 1 - r exact).  The panel is the first one (from the
// respective end) whose running sum reaches the target.
template <class F>
double invert_cdf(const F& f, const CdfPanels& c, double r, double rc) {
  if (!(c.tot > 0.0)) return 0.0;
  const size_t n = c.ps.size();
  if (r <= 0.5) {
    const double target = r * c.tot;
    const size_t k = std::lower_bound(c.lo.begin(), c.lo.end(), target) - c.lo.begin();
    if (k == n) return c.ps.back().b;
    const Panel& p = c.ps[k];
    return invert_in_panel(f, p.a, p.b, target - (k > 0 ? c.lo[k - 1] : 0.0), p.val());
  }
  // from the top: find x with int_x^end f = rc * tot
  const double target = rc * c.tot;
  // hi is non-increasing in k: the largest k with hi[k] >= target
  size_t lo = 0, hi = n;
  while (lo < hi) {
    const size_t mid = (lo + hi) / 2;
    if (c.hi[mid] >= target) lo = mid + 1; else hi = mid;
  }
  if (lo == 0) return c.ps.front().a;
  const size_t k = lo - 1;
  const Panel& p = c.ps[k];
  // int_{p.a}^{x} f = p.val - (target - cum), cum = sum of the panels above k
  const double cum = k + 1 < n ? c.hi[k + 1] : 0.0;
  return invert_in_panel(f, p.a, p.b, p.val() - (target - cum), p.val());
}

template <class F>
double invert_cdf(const F& f, const std::vector<double>& breaks, double r, double rc,
                  double* total_out) {
  const CdfPanels c = cdf_panels(f, breaks);
  if (total_out) *total_out = c.tot;
  return invert_cdf(f, c, r, rc);
}

// Inverse CDF of the emission spectrum: returns delta and 1 - delta.
void sample_rad(double chi, double r, double rc, bool def, double* d, double* omd) {
  const double v = invert_cdf(RadVar{chi, def}, rad_breaks(chi), r, rc, nullptr);
  const double z = 1.5 * chi * v * v * v;
  *d = z / (1.0 + z);
  *omd = 1.0 / (1.0 + z);
}

// Inverse CDF of the pair spectrum on (0, 1/2], extended by symmetry.
void sample_pair(double chi, double r, double rc, bool def, double* xi, double* omx) {
  if (r <= 0.5) {
    const double x = invert_cdf(PairVar{chi, def}, pair_breaks(chi), 2.0 * r, 1.0 - 2.0 * r, nullptr);
    *xi = x;
    *omx = 1.0 - x;
  } else {
    const double x = invert_cdf(PairVar{chi, def}, pair_breaks(chi), 2.0 * rc, 1.0 - 2.0 * rc, nullptr);
    *xi = 1.0 - x;
    *omx = x;
  }
}

// ---------------------------------------------------------------------------
// chi (Calculate chi in Alg. 1):
//   lepton: chi = sqrt((gamma E + p x B)^2 - (p.E)^2), gamma = sqrt(1+p^2)
//   photon: chi = sqrt((eps E + k x B)^2 - (k.E)^2),   eps = |k|
// ---------------------------------------------------------------------------
inline void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

double chi_of(const double p[3], double energy, const double E[3], const double B[3]) {
  double pxb[3];
  cross(p, B, pxb);
  double a[3];
  for (int i = 0; i < 3; ++i) a[i] = energy * E[i] + pxb[i];
  const double b = dot(p, E);
  const double c2 = dot(a, a) - b * b;
  return c2 > 0.0 ? std::sqrt(c2) : 0.0;
}

// Boris rotation/acceleration over h for charge q (the textbook scheme of
// Boris 1970: half electric kick, magnetic rotation, half electric kick).
void boris(double p[3], double q, const double E[3], const double B[3], double h) {
  double um[3];
  for (int i = 0; i < 3; ++i) um[i] = p[i] + 0.5 * q * h * E[i];
  const double gm = std::sqrt(1.0 + dot(um, um));
  double t[3];
  for (int i = 0; i < 3; ++i) t[i] = 0.5 * q * h * B[i] / gm;
  const double f = 2.0 / (1.0 + dot(t, t));
  double s[3];
  for (int i = 0; i < 3; ++i) s[i] = f * t[i];
  double c[3];
  cross(um, t, c);
  double up[3];
  for (int i = 0; i < 3; ++i) up[i] = um[i] + c[i];
  cross(up, s, c);
  for (int i = 0; i < 3; ++i) p[i] = um[i] + c[i] + 0.5 * q * h * E[i];
}

}  // namespace

// ===========================================================================
// C interface (ctypes).
// ===========================================================================
extern "C" {

// Per-species particle store, FP64.  state is [capacity x 9]:
// px py pz x y z w tau t_birth.  root is the field reference of the particle
// (species << 30 | index into that species' field array).
typedef struct {
  double* state;
  uint64_t* id;
  int32_t* root;
  uint8_t* alive;
  int32_t* nev;
  int64_t count, capacity;
} orc_species;

typedef struct {
  const double* f;  // [n x 6]: ex ey ez bx by bz
  int64_t stride;   // 1: per particle, 0: one value for all
} orc_fields;

typedef struct {
  int32_t emission, pair, push, positions;
  int64_t max_events;
  double gamma_min;  // leptons below this Lorentz factor do not emit
} orc_cfg;

typedef struct {
  int64_t n_emit, n_pair, n_new[3], n_rounds, max_events, overflow, capped;
} orc_stats;

void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox4x32_10(ctr, key, out); }

void orc_philox_stream(uint64_t seed, const uint64_t* id, const uint32_t* step, const uint32_t* j,
                       int64_t n, uint32_t* out) {
  for (int64_t i = 0; i < n; ++i) draw(seed, id[i], step[i], j[i], out + 4 * i);
}

double orc_alpha() { return kAlpha; }

double orc_bessel_k(double nu, double x, int def) {
  if (def) return std::exp(-x) * bessel_k_scaled_def(nu, x);
  if (std::fabs(nu - 2.0 / 3.0) < 1e-15) return k23(x, false);
  return std::exp(-x) * bessel_k_scaled_def(nu, x);
}

double orc_bessel_ki(double nu, double x, int def) {
  if (!def && std::fabs(nu - 1.0 / 3.0) < 1e-15) return ki13(x, false);
  return std::exp(-x) * bessel_ki_scaled_def(nu, x);
}

double orc_spec_rad(double chi, double d, int def) { return spec_rad(chi, d, 1.0 - d, def != 0); }
double orc_spec_pair(double chi, double xi, int def) { return spec_pair(chi, xi, 1.0 - xi, def != 0); }

void orc_spec_rad_many(const double* chi, const double* d, int64_t n, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = spec_rad(chi[i], d[i], 1.0 - d[i], false);
}

void orc_spec_pair_many(const double* chi, const double* xi, int64_t n, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = spec_pair(chi[i], xi[i], 1.0 - xi[i], false);
}

// W * gamma / alpha and W * eps / alpha
double orc_rate_rad(double chi, int def) { return rate_rad_reduced(chi, def != 0); }
double orc_rate_pair(double chi, int def) { return rate_pair_reduced(chi, def != 0); }

void orc_rate_rad_many(const double* chi, int64_t n, double* out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) out[i] = rate_rad_reduced(chi[i], false);
}
void orc_rate_pair_many(const double* chi, int64_t n, double* out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) out[i] = rate_pair_reduced(chi[i], false);
}

// CDF of the emission spectrum at delta: int_0^delta / int_0^1.
double orc_cdf_rad(double chi, double d, int def) {
  const bool df = def != 0;
  const double tot = rate_rad_reduced(chi, df);
  // delta -> v: z = d/(1-d), y = 2z/(3chi), v = y^{1/3}
  const double z = d / (1.0 - d);
  const double v = std::cbrt(2.0 * z / (3.0 * chi));
  std::vector<double> br = rad_breaks(chi);
  std::vector<double> b2{0.0};
  for (double x : br)
    if (x > 0.0 && x < v) b2.push_back(x);
  b2.push_back(v);
  return quad(RadVar{chi, df}, b2, kRtol, kRtol * tot) / tot;
}

double orc_cdf_pair(double chi, double xi, int def) {
  const bool df = def != 0;
  const double tot = rate_pair_reduced(chi, df);
  std::vector<double> br = pair_breaks(chi);
  // pair_breaks covers (0, 1/2]; extend to 1 by mirroring
  std::vector<double> full;
  for (double x : br) full.push_back(x);
  for (double x : br) full.push_back(1.0 - x);
  std::sort(full.begin(), full.end());
  full.erase(std::unique(full.begin(), full.end()), full.end());
  std::vector<double> b2;
  for (double x : full)
    if (x < xi) b2.push_back(x);
  b2.push_back(xi);
  return quad(PairVar{chi, df}, b2, kRtol, kRtol * tot) / tot;
}

// Sampling from raw 32-bit uniforms k: r = (k + 1/2) 2^-32.
void orc_sample_rad(const double* chi, const uint32_t* k, int64_t n, double* d, double* omd) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) sample_rad(chi[i], u01(k[i]), u01c(k[i]), false, d + i, omd + i);
}

void orc_sample_pair(const double* chi, const uint32_t* k, int64_t n, double* xi, double* omx) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) sample_pair(chi[i], u01(k[i]), u01c(k[i]), false, xi + i, omx + i);
}

// Emission draws on a chi grid: for chi[i] the spectrum's panels are built
// once and r[i*k + j], j < k, are inverted (rc = 1 - r exact).  Same values as
// orc_sample_rad_r with the fast tier.
void orc_sample_rad_grid(const double* chi, int64_t m, const double* r, const double* rc, int64_t k, double* d,
                         double* omd) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < m; ++i) {
    const RadVar f{chi[i], false};
    const CdfPanels c = cdf_panels(f, rad_breaks(chi[i]));
    for (int64_t j = i * k; j < (i + 1) * k; ++j) {
      const double v = invert_cdf(f, c, r[j], rc[j]);
      const double z = 1.5 * chi[i] * v * v * v;
      d[j] = z / (1.0 + z);
      omd[j] = 1.0 / (1.0 + z);
    }
  }
}

// Same with a general r in (0,1) (rc = 1 - r), definitions or fast tier.
void orc_sample_rad_r(double chi, double r, double rc, int def, double* d, double* omd) {
  sample_rad(chi, r, rc, def != 0, d, omd);
}
void orc_sample_pair_r(double chi, double r, double rc, int def, double* xi, double* omx) {
  sample_pair(chi, r, rc, def != 0, xi, omx);
}

double orc_chi(const double* p, double energy, const double* E, const double* B) { return chi_of(p, energy, E, B); }

void orc_boris(double* p, double q, const double* E, const double* B, double h) { boris(p, q, E, B, h); }

// Optical depth for particles with tau < 0: tau = -ln(u0), u0 from counter
// j = 0xFFFFFFFF (reserved for initial draws).
void orc_init_tau(orc_species* s, uint64_t seed, uint32_t step) {
  for (int64_t i = 0; i < s->count; ++i) {
    double* st = s->state + 9 * i;
    if (st[7] < 0.0) {
      uint32_t u[4];
      draw(seed, s->id[i], step, 0xFFFFFFFFu, u);
      st[7] = -std::log(u01(u[0]));
    }
  }
}

}  // extern "C"

namespace {

struct Child {
  int sp;
  double p[3], x[3], w, tau, tb;
  uint64_t id;
  int32_t root;
};

struct Ctx {
  const orc_fields* f;
  double dt;
  uint64_t seed;
  uint32_t step;
  const orc_cfg* cfg;
};

struct Local {
  std::vector<Child> kids;
  int64_t n_emit = 0, n_pair = 0, max_events = 0;
  bool capped = false;
};

void field_of(const Ctx& c, int32_t root, double E[3], double B[3]) {
  const int sp = (int)((uint32_t)root >> 30);
  const int64_t idx = (int64_t)((uint32_t)root & 0x3FFFFFFFu);
  const double* fr = c.f[sp].f + 6 * (c.f[sp].stride ? idx : 0);
  for (int i = 0; i < 3; ++i) { E[i] = fr[i]; B[i] = fr[3 + i]; }
}

// Alg. 1 for a lepton of charge q, with the optical depth carried across
// subcycles (state s = px py pz x y z w tau t_birth).
void push_lepton(const Ctx& c, double* s, uint64_t id, int32_t root, double q, int32_t* nev_out,
                 Local& L) {
  double E[3], B[3];
  field_of(c, root, E, B);
  double p[3] = {s[0], s[1], s[2]};
  double x[3] = {s[3], s[4], s[5]};
  const double w = s[6];
  double tau = s[7];
  double t = s[8];
  const double dt = c.dt;
  uint32_t j = 0;
  bool capped = false;
  auto advance = [&](double h) {
    if (c.cfg->push) boris(p, q, E, B, h);
    if (c.cfg->positions) {
      const double g = std::sqrt(1.0 + dot(p, p));
      for (int i = 0; i < 3; ++i) x[i] += p[i] / g * h;
    }
  };
  while (t < dt) {
    const double g = std::sqrt(1.0 + dot(p, p));
    const double chi = chi_of(p, g, E, B);
    const double W = (c.cfg->emission && !capped && g >= c.cfg->gamma_min)
                         ? kAlpha / g * rate_rad_reduced(chi, false)
                         : 0.0;
    const double rem = dt - t;
    if (!(W > 0.0) || tau > W * rem) {  // no event before the end of the step
      tau -= W * rem;
      advance(rem);
      t = dt;
      break;
    }
    double h = tau / W;  // the optical depth is used up after h
    if (h > rem) h = rem;
    advance(h);
    t += h;
    uint32_t u[4];
    draw(c.seed, id, c.step, j, u);
    const double ge = std::sqrt(1.0 + dot(p, p));
    const double chi_e = chi_of(p, ge, E, B);  // the particle as it is at the event
    double d, omd;
    sample_rad(chi_e, u01(u[0]), u01c(u[0]), false, &d, &omd);
    Child ch;
    ch.sp = 2;
    for (int i = 0; i < 3; ++i) {
      ch.p[i] = d * p[i];  // collinear recoil: k = delta p, p -> (1 - delta) p
      p[i] = omd * p[i];
      ch.x[i] = x[i];
    }
    tau = -std::log(u01(u[1]));
    uint32_t v[4];
    draw(c.seed, id, c.step, j | 0x80000000u, v);
    ch.id = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
    ch.w = w;
    ch.tau = -std::log(u01(u[2]));
    ch.tb = t;
    ch.root = root;
    L.kids.push_back(ch);
    L.n_emit++;
    ++j;
    if ((int64_t)j >= c.cfg->max_events) {
      capped = true;
      L.capped = true;
    }
  }
  s[0] = p[0]; s[1] = p[1]; s[2] = p[2];
  s[3] = x[0]; s[4] = x[1]; s[5] = x[2];
  s[7] = tau;
  if (nev_out) *nev_out = (int32_t)j;
  if ((int64_t)j > L.max_events) L.max_events = j;
}

// The photon counterpart (PhotonPush in Alg. 2): pair rate, straight-line
// advance, and the photon is removed at its first event.
void push_photon(const Ctx& c, double* s, uint64_t id, int32_t root, uint8_t* alive, int32_t* nev_out,
                 Local& L) {
  double E[3], B[3];
  field_of(c, root, E, B);
  const double k[3] = {s[0], s[1], s[2]};
  double x[3] = {s[3], s[4], s[5]};
  const double w = s[6];
  double tau = s[7];
  double t = s[8];
  const double dt = c.dt;
  const double eps = std::sqrt(dot(k, k));
  int32_t ev = 0;
  auto advance = [&](double h) {
    if (c.cfg->positions && eps > 0.0)
      for (int i = 0; i < 3; ++i) x[i] += k[i] / eps * h;
  };
  while (t < dt) {
    const double chi = chi_of(k, eps, E, B);
    // below eps = 2 (two electron masses) no pair can be made
    const double W = (c.cfg->pair && eps >= 2.0) ? kAlpha / eps * rate_pair_reduced(chi, false) : 0.0;
    const double rem = dt - t;
    if (!(W > 0.0) || tau > W * rem) {
      tau -= W * rem;
      advance(rem);
      t = dt;
      break;
    }
    double h = tau / W;
    if (h > rem) h = rem;
    advance(h);
    t += h;
    uint32_t u[4];
    draw(c.seed, id, c.step, 0u, u);
    double xi, omx;
    sample_pair(chi, u01(u[0]), u01c(u[0]), false, &xi, &omx);
    uint32_t v[4];
    draw(c.seed, id, c.step, 0x80000000u, v);
    Child e, q;
    e.sp = 0;
    q.sp = 1;
    for (int i = 0; i < 3; ++i) {
      e.p[i] = xi * k[i];  // the electron takes xi of the photon momentum
      q.p[i] = omx * k[i];
      e.x[i] = q.x[i] = x[i];
    }
    e.id = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
    q.id = (uint64_t)v[2] | ((uint64_t)v[3] << 32);
    e.tau = -std::log(u01(u[2]));
    q.tau = -std::log(u01(u[3]));
    e.w = q.w = w;
    e.tb = q.tb = t;
    e.root = q.root = root;
    L.kids.push_back(e);
    L.kids.push_back(q);
    L.n_pair++;
    *alive = 0;
    ev = 1;
    break;
  }
  s[3] = x[0]; s[4] = x[1]; s[5] = x[2];
  s[7] = tau;
  if (nev_out) *nev_out = ev;
  if (ev > L.max_events) L.max_events = ev;
}

// Processes particles [lo, hi) of store `s` (species sp) in parallel and
// appends their children in index order (then event order).
void run_range(const Ctx& c, orc_species* app, orc_stats* st, orc_species& s, int sp, int64_t lo,
               int64_t hi, bool main_store) {
  if (hi <= lo) return;
  std::vector<Local> loc(hi - lo);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = lo; i < hi; ++i) {
    Local& L = loc[i - lo];
    const int32_t root = main_store ? (int32_t)(((uint32_t)sp << 30) | (uint32_t)i) : s.root[i];
    int32_t* nev = s.nev ? s.nev + i : nullptr;
    if (sp < 2) {
      push_lepton(c, s.state + 9 * i, s.id[i], root, sp == 0 ? -1.0 : 1.0, nev, L);
    } else {
      if (s.alive && !s.alive[i]) continue;
      uint8_t dummy = 1;
      push_photon(c, s.state + 9 * i, s.id[i], root, s.alive ? s.alive + i : &dummy, nev, L);
    }
  }
  for (Local& L : loc) {
    st->n_emit += L.n_emit;
    st->n_pair += L.n_pair;
    st->max_events = std::max(st->max_events, L.max_events);
    if (L.capped) st->capped = 1;
    for (const Child& ch : L.kids) {
      orc_species& a = app[ch.sp];
      st->n_new[ch.sp]++;
      if (a.count >= a.capacity) {
        st->overflow = 1;
        a.count++;
        continue;
      }
      double* r = a.state + 9 * a.count;
      r[0] = ch.p[0]; r[1] = ch.p[1]; r[2] = ch.p[2];
      r[3] = ch.x[0]; r[4] = ch.x[1]; r[5] = ch.x[2];
      r[6] = ch.w; r[7] = ch.tau; r[8] = ch.tb;
      a.id[a.count] = ch.id;
      a.root[a.count] = ch.root;
      a.alive[a.count] = 1;
      if (a.nev) a.nev[a.count] = 0;
      a.count++;
    }
  }
}

}  // namespace

extern "C" {

// One global step of the whole ensemble (Alg. 2 applied to every particle):
// rounds of "all pending leptons (electrons, then positrons, each in index
// order), then all pending photons (including those just emitted)", until a
// round creates nothing.  Children go to the append store in creation order.
// main[s].state[8] (t_birth) is the start time of each main particle (0).
int orc_step(orc_species* main, const orc_fields* f, orc_species* app, double dt, uint64_t seed,
             uint32_t step, const orc_cfg* cfg, orc_stats* st) {
  std::memset(st, 0, sizeof(*st));
  Ctx c{f, dt, seed, step, cfg};
  for (int s = 0; s < 3; ++s) app[s].count = 0;
  auto stored = [&](int sp) { return std::min(app[sp].count, app[sp].capacity); };
  // round 0: the main store, then the photons it emitted
  run_range(c, app, st, main[0], 0, 0, main[0].count, true);
  run_range(c, app, st, main[1], 1, 0, main[1].count, true);
  run_range(c, app, st, main[2], 2, 0, main[2].count, true);
  int64_t ph_lo = stored(2);
  run_range(c, app, st, app[2], 2, 0, ph_lo, false);
  int64_t lep_lo = 0, lep_hi = stored(0);
  int64_t rounds = 1;
  while (!st->overflow && lep_hi > lep_lo) {
    run_range(c, app, st, app[0], 0, lep_lo, lep_hi, false);
    run_range(c, app, st, app[1], 1, lep_lo, lep_hi, false);
    const int64_t ph_hi = stored(2);
    run_range(c, app, st, app[2], 2, ph_lo, ph_hi, false);
    ph_lo = ph_hi;
    lep_lo = lep_hi;
    lep_hi = stored(0);
    ++rounds;
  }
  st->n_rounds = rounds;
  return st->overflow ? 2 : (st->capped ? 5 : 0);
}

// Merge: drop photons with alive = 0 (stable), then append the surviving
// children of each species after the survivors.
int orc_merge(orc_species* main, const orc_species* app) {
  for (int sp = 0; sp < 3; ++sp) {
    orc_species& m = main[sp];
    int64_t n = 0;
    for (int64_t i = 0; i < m.count; ++i) {
      if (m.alive && !m.alive[i]) continue;
      if (n != i) {
        std::memcpy(m.state + 9 * n, m.state + 9 * i, 9 * sizeof(double));
        m.id[n] = m.id[i];
        if (m.alive) m.alive[n] = 1;
      }
      ++n;
    }
    const orc_species& a = app[sp];
    for (int64_t i = 0; i < a.count; ++i) {
      if (a.alive && !a.alive[i]) continue;
      if (n >= m.capacity) return 2;
      std::memcpy(m.state + 9 * n, a.state + 9 * i, 9 * sizeof(double));
      m.state[9 * n + 8] = 0.0;
      m.id[n] = a.id[i];
      if (m.alive) m.alive[n] = 1;
      ++n;
    }
    m.count = n;
  }
  return 0;
}

}  // extern "C"
