// host_simd.cpp -- a host-CPU baseline of the per-macroparticle event
// generator, organised as the paper's CPU implementation is (Sec. 4.3,
// Algorithm 3): particles are processed in chunks of a compile-time size; each
// trip over a chunk runs the physics of every particle still in flight in one
// vectorisable loop, the random numbers and appends in separate loops, and then
// moves the particles that reached the end of the step out of the way so that
// the next trip runs over the rest only.  Chunks are spread over OpenMP threads.
// Generations follow Algorithm 2 (leptons, then photons, in rounds).
//
// It is a measurement baseline, not part of the GPU library: it shares no code
// with it and is only run by the benchmark's CPU leg and its own tests.  Its
// rate and inverse-CDF tables are node values given by the caller; the
// interpolation is its own (cubic Lagrange in ln chi for ln W, and in
// (ln chi, logit r) for the sampled fractions).  The random stream is the one
// the method fixes (Philox4x32-10 keyed by the seed, counter = (id, step, j)),
// so its results can be compared particle by particle with any other
// implementation of the same stream.
//
// Built with -O3 -ffast-math -fopenmp so that log, exp and sqrt in the chunk
// loops map to vector library calls, once per instruction set (x86-64-v4 with
// AVX-512, x86-64-v3 with AVX2 and FMA, baseline x86-64); the loader picks the
// best one the host supports.

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#define HS_INLINE __attribute__((always_inline)) inline
#ifndef HS_ISA
#define HS_ISA "x86-64"
#endif

namespace {

constexpr int kChunk = 64;                  // particles per chunk (Algorithm 3's compile-time size)
constexpr double kAlpha = 7.2973525693e-3;  // fine-structure constant (CODATA 2018)

// ---------------------------------------------------------------------------- Philox4x32-10
struct U4 {
  uint32_t v[4];
};

HS_INLINE U4 philox(uint64_t seed, uint64_t id, uint32_t step, uint32_t j) {
  uint32_t c0 = (uint32_t)id, c1 = (uint32_t)(id >> 32), c2 = step, c3 = j;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma GCC unroll 10
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = (uint64_t)0xD2511F53u * c0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)b;
    c3 = (uint32_t)a;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{{c0, c1, c2, c3}};
}

// -ln u for u = (k + 1/2) 2^-32, in FP64
HS_INLINE double neg_log_u(uint32_t k) { return -std::log(((double)k + 0.5) * 0x1p-32); }
// logit r = ln(r / (1 - r)) with 1 - r = (~k + 1/2) 2^-32 exact
HS_INLINE double logit_u(uint32_t k) { return std::log((double)k + 0.5) - std::log((double)(~k) + 0.5); }

// ---------------------------------------------------------------------------- tables
template <typename T>
struct Tables {
  int nr = 0;
  T s0 = 0, inv_hr = 0;
  std::vector<T> lnr[2];  // ln of the reduced rate (W * energy / alpha) at s = s0 + i h
  int rows[2] = {0, 0}, cols[2] = {0, 0};
  T qs0[2], inv_qhs[2], qx0[2], inv_qhx[2];
  std::vector<T> q[2];  // [rows][cols]
};

// cubic Lagrange weights at fractional position t in [0, 1] for nodes -1, 0, 1, 2
template <typename T>
HS_INLINE void lag4(T t, T w[4]) {
  const T tm1 = t - T(1), tm2 = t - T(2), tp1 = t + T(1);
  w[0] = -t * tm1 * tm2 * T(1.0 / 6.0);
  w[1] = tp1 * tm1 * tm2 * T(0.5);
  w[2] = -tp1 * t * tm2 * T(0.5);
  w[3] = tp1 * t * tm1 * T(1.0 / 6.0);
}

// first of the four nodes and the fractional position, clamped to the table
template <typename T>
HS_INLINE int node4(T u, int n, T& t) {
  const T um = std::min(std::max(u, T(1)), T(n - 2) - T(1e-4));
  const int i = (int)um;
  t = um - (T)i;
  return i - 1;
}

// One rate table as the loops see it (hoisted out of them).
template <typename T>
struct RateRef {
  const T* __restrict v;
  int n;
  T s0, inv_h;
};

template <typename T>
RateRef<T> rate_ref(const Tables<T>& tb, int proc) {
  return RateRef<T>{tb.lnr[proc].data(), tb.nr, tb.s0, tb.inv_hr};
}

template <typename T>
HS_INLINE T rate_reduced(const RateRef<T>& R, T s) {
  T t;
  const int i = node4((s - R.s0) * R.inv_h, R.n, t);
  T w[4];
  lag4(t, w);
  const T* __restrict v = R.v;
  return std::exp(w[0] * v[i] + w[1] * v[i + 1] + w[2] * v[i + 2] + w[3] * v[i + 3]);
}

// One inverse-CDF grid as the loops see it.
template <typename T>
struct GridRef {
  const T* __restrict q;
  int rows, cols;
  T s0, inv_hs, x0, inv_hx;
};

template <typename T>
GridRef<T> grid_ref(const Tables<T>& tb, int proc) {
  return GridRef<T>{tb.q[proc].data(), tb.rows[proc], tb.cols[proc], tb.qs0[proc], tb.inv_qhs[proc], tb.qx0[proc],
                    tb.inv_qhx[proc]};
}

template <typename T>
HS_INLINE T q_interp(const GridRef<T>& G, T s, T x) {
  T ts, tx;
  const int r = node4((s - G.s0) * G.inv_hs, G.rows, ts);
  const int c = node4((x - G.x0) * G.inv_hx, G.cols, tx);
  T ws[4], wx[4];
  lag4(ts, ws);
  lag4(tx, wx);
  const int nc = G.cols;
  const T* __restrict q = G.q;
  T acc = 0;
#pragma GCC unroll 4
  for (int a = 0; a < 4; ++a) {
    const int o = (r + a) * nc + c;  // the grids hold well under 2^31 values
    acc += ws[a] * (wx[0] * q[o] + wx[1] * q[o + 1] + wx[2] * q[o + 2] + wx[3] * q[o + 3]);
  }
  return acc;
}

// ---------------------------------------------------------------------------- particles
template <typename T>
struct Species {
  T *px, *py, *pz, *x, *y, *z;
  float* w;
  double* tau;
  uint64_t* id;
  uint8_t* alive;
  int32_t* nev;
  double* t_birth;  // appended particles only
  uint32_t* root;   // appended particles only
  int64_t count, capacity;
};

template <typename T>
struct Fields {
  const T *ex, *ey, *ez, *bx, *by, *bz;
  int64_t stride;
};

struct Cfg {
  int32_t emission, pair, push, positions;
  double gamma_min;
  int64_t max_events;
};

template <typename T>
struct Child {
  T p[3], x[3];
  double tau, tb;
  uint64_t id;
  float w;
  uint32_t root;
  int32_t parent, sp;  // lane of the parent in its chunk, species
};

template <typename T>
struct Ctx {
  const Tables<T>* tb;
  const Fields<T>* f;
  const Cfg* cfg;
  double dt;
  uint64_t seed;
  uint32_t step;
};

// Lane data of one chunk, structure of arrays.  Lanes [0, live) are still in
// flight; finished lanes are swapped behind them.
template <typename T>
struct Chunk {
  T px[kChunk], py[kChunk], pz[kChunk], x[kChunk], y[kChunk], z[kChunk];
  T ex[kChunk], ey[kChunk], ez[kChunk], bx[kChunk], by[kChunk], bz[kChunk];
  double tau[kChunk], t[kChunk];
  uint64_t id[kChunk];
  float w[kChunk];
  uint32_t root[kChunk];
  int32_t lane[kChunk], nev[kChunk];
  T gcut[kChunk];  // emission threshold in gamma: gamma_min, or above any gamma once max_events is reached
  // per trip: ln chi and the rate of each lane in flight
  T chi[kChunk], W[kChunk];
  int32_t ev[kChunk];
};

template <typename T>
inline void swap_lanes(Chunk<T>& c, int a, int b) {
  std::swap(c.px[a], c.px[b]); std::swap(c.py[a], c.py[b]); std::swap(c.pz[a], c.pz[b]);
  std::swap(c.x[a], c.x[b]); std::swap(c.y[a], c.y[b]); std::swap(c.z[a], c.z[b]);
  std::swap(c.ex[a], c.ex[b]); std::swap(c.ey[a], c.ey[b]); std::swap(c.ez[a], c.ez[b]);
  std::swap(c.bx[a], c.bx[b]); std::swap(c.by[a], c.by[b]); std::swap(c.bz[a], c.bz[b]);
  std::swap(c.tau[a], c.tau[b]); std::swap(c.t[a], c.t[b]); std::swap(c.id[a], c.id[b]);
  std::swap(c.w[a], c.w[b]); std::swap(c.root[a], c.root[b]); std::swap(c.lane[a], c.lane[b]);
  std::swap(c.nev[a], c.nev[b]); std::swap(c.gcut[a], c.gcut[b]); std::swap(c.ev[a], c.ev[b]);
}

// Moves lanes whose flag is 0 behind the others (in linear time); returns
// the number of lanes left in flight.
template <typename T>
inline int compact(Chunk<T>& c, int live, const int32_t* keep) {
  int lo = 0, hi = live - 1;
  int32_t k[kChunk];
  std::memcpy(k, keep, sizeof(int32_t) * live);
  while (true) {
    while (lo <= hi && k[lo]) ++lo;
    while (lo <= hi && !k[hi]) --hi;
    if (lo >= hi) break;
    swap_lanes(c, lo, hi);
    std::swap(k[lo], k[hi]);
    ++lo;
    --hi;
  }
  return lo;
}

template <typename T>
void load_chunk(const Ctx<T>& C, const Species<T>& s, int sp, bool from_main, int64_t lo, int n, Chunk<T>& c) {
  for (int l = 0; l < n; ++l) {
    const int64_t i = lo + l;
    c.px[l] = s.px[i]; c.py[l] = s.py[i]; c.pz[l] = s.pz[i];
    if (C.cfg->positions) {
      c.x[l] = s.x[i]; c.y[l] = s.y[i]; c.z[l] = s.z[i];
    } else {
      c.x[l] = c.y[l] = c.z[l] = T(0);
    }
    c.tau[l] = s.tau[i];
    c.t[l] = from_main ? 0.0 : s.t_birth[i];
    c.id[l] = s.id[i];
    c.w[l] = s.w[i];
    c.root[l] = from_main ? (((uint32_t)sp << 30) | (uint32_t)i) : s.root[i];
    c.lane[l] = l;
    c.nev[l] = 0;
    c.gcut[l] = (T)C.cfg->gamma_min;
    const int fs = (int)(c.root[l] >> 30);
    const Fields<T>& F = C.f[fs];
    const int64_t fi = F.stride ? (int64_t)(c.root[l] & 0x3FFFFFFFu) : 0;
    c.ex[l] = F.ex[fi]; c.ey[l] = F.ey[fi]; c.ez[l] = F.ez[fi];
    c.bx[l] = F.bx[fi]; c.by[l] = F.by[fi]; c.bz[l] = F.bz[fi];
  }
}

template <typename T>
void store_chunk(const Ctx<T>& C, Species<T>& s, int64_t lo, int n, const Chunk<T>& c) {
  for (int l = 0; l < n; ++l) {
    const int64_t i = lo + c.lane[l];
    s.px[i] = c.px[l]; s.py[i] = c.py[l]; s.pz[i] = c.pz[l];
    if (C.cfg->positions) {
      s.x[i] = c.x[l]; s.y[i] = c.y[l]; s.z[i] = c.z[l];
    }
    s.tau[i] = c.tau[l];
    if (s.nev) s.nev[i] = c.nev[l];
  }
}

// chi^2 = |e E + p x B|^2 - (p . E)^2, clamped at 0
template <typename T>
HS_INLINE T chi2_of(T px, T py, T pz, T e, T ex, T ey, T ez, T bx, T by, T bz) {
  const T ax = e * ex + (py * bz - pz * by);
  const T ay = e * ey + (pz * bx - px * bz);
  const T az = e * ez + (px * by - py * bx);
  const T b = px * ex + py * ey + pz * ez;
  return std::max(ax * ax + ay * ay + az * az - b * b, T(0));
}

template <typename T>
HS_INLINE void boris(T& px, T& py, T& pz, T q, T ex, T ey, T ez, T bx, T by, T bz, T h) {
  const T k = T(0.5) * q * h;
  const T ux = px + k * ex, uy = py + k * ey, uz = pz + k * ez;
  const T gm = std::sqrt(T(1) + ux * ux + uy * uy + uz * uz);
  const T tx = k * bx / gm, ty = k * by / gm, tz = k * bz / gm;
  const T f = T(2) / (T(1) + tx * tx + ty * ty + tz * tz);
  const T vx = ux + (uy * tz - uz * ty), vy = uy + (uz * tx - ux * tz), vz = uz + (ux * ty - uy * tx);
  px = ux + (vy * f * tz - vz * f * ty) + k * ex;
  py = uy + (vz * f * tx - vx * f * tz) + k * ey;
  pz = uz + (vx * f * ty - vy * f * tx) + k * ez;
}

// Algorithm 3 for leptons of charge q: trips over the chunk until every
// particle reached the end of the step.
template <typename T, bool push, bool positions>
void lepton_chunk(const Ctx<T>& C, Chunk<T>& c, int n, T q, std::vector<Child<T>>& kids, int64_t& n_emit,
                  bool& any_capped) {
  const RateRef<T> R = rate_ref(*C.tb, 0);
  const GridRef<T> G = grid_ref(*C.tb, 0);
  const Cfg& cfg = *C.cfg;
  const double dt = C.dt;
  const bool emission = cfg.emission != 0;
  int live = n;
  while (live > 0) {
    // 1. physics of every particle in flight: chi and the rate (vector loop),
    //    then the event decision and the advance (vector loop)
#pragma omp simd
    for (int l = 0; l < live; ++l) {
      const T g = std::sqrt(T(1) + c.px[l] * c.px[l] + c.py[l] * c.py[l] + c.pz[l] * c.pz[l]);
      const T c2 = chi2_of(c.px[l], c.py[l], c.pz[l], g, c.ex[l], c.ey[l], c.ez[l], c.bx[l], c.by[l], c.bz[l]);
      const bool on = emission && g >= c.gcut[l] && c2 > T(0);
      c.chi[l] = T(0.5) * std::log(std::max(c2, T(1e-30)));  // ln chi
      c.W[l] = on ? T(kAlpha) / g : T(0);                    // the rate's prefactor
    }
#pragma omp simd
    for (int l = 0; l < live; ++l) c.W[l] *= rate_reduced(R, c.chi[l]);
#pragma omp simd
    for (int l = 0; l < live; ++l) {
      const T W = c.W[l];
      const double rem = dt - c.t[l];
      const double Wr = (double)W * rem;
      const int ev = (W > T(0)) && !(c.tau[l] > Wr);
      double h = ev ? c.tau[l] / (double)W : rem;
      if (h > rem) h = rem;
      c.tau[l] = ev ? c.tau[l] : c.tau[l] - Wr;
      c.t[l] = ev ? c.t[l] + h : dt;
      const T hh = (T)h;
      if (push) boris(c.px[l], c.py[l], c.pz[l], q, c.ex[l], c.ey[l], c.ez[l], c.bx[l], c.by[l], c.bz[l], hh);
      if (positions) {
        const T gi = T(1) / std::sqrt(T(1) + c.px[l] * c.px[l] + c.py[l] * c.py[l] + c.pz[l] * c.pz[l]);
        c.x[l] += c.px[l] * gi * hh;
        c.y[l] += c.py[l] * gi * hh;
        c.z[l] += c.pz[l] * gi * hh;
      }
      c.ev[l] = ev;
    }
    // 2. events: draws, the sampled fraction, recoil (a vector loop over the
    //    lanes with events, then a scalar loop for the appends)
    int ne = 0;
    int32_t idx[kChunk];
    for (int l = 0; l < live; ++l)
      if (c.ev[l]) idx[ne++] = l;
    T dlt[kChunk], omd[kChunk];
    double tnew[kChunk], tch[kChunk];
    uint64_t cid[kChunk];
#pragma omp simd
    for (int e = 0; e < ne; ++e) {
      const int l = idx[e];
      const U4 u = philox(C.seed, c.id[l], C.step, (uint32_t)c.nev[l]);
      const U4 v = philox(C.seed, c.id[l], C.step, (uint32_t)c.nev[l] | 0x80000000u);
      T s = c.chi[l];  // ln chi at the start of the sub-interval
      if (push) {      // the particle has moved: chi at the event point
        const T g = std::sqrt(T(1) + c.px[l] * c.px[l] + c.py[l] * c.py[l] + c.pz[l] * c.pz[l]);
        const T c2 = chi2_of(c.px[l], c.py[l], c.pz[l], g, c.ex[l], c.ey[l], c.ez[l], c.bx[l], c.by[l], c.bz[l]);
        s = T(0.5) * std::log(std::max(c2, T(1e-30)));
      }
      const T z = q_interp(G, s, (T)logit_u(u.v[0])) + s;  // logit of the emitted fraction
      dlt[e] = T(1) / (T(1) + std::exp(-z));
      omd[e] = T(1) / (T(1) + std::exp(z));
      tnew[e] = neg_log_u(u.v[1]);
      tch[e] = neg_log_u(u.v[2]);
      cid[e] = (uint64_t)v.v[0] | ((uint64_t)v.v[1] << 32);
    }
    for (int e = 0; e < ne; ++e) {
      const int l = idx[e];
      const T d = dlt[e], od = omd[e];
      Child<T> ch;
      ch.p[0] = d * c.px[l]; ch.p[1] = d * c.py[l]; ch.p[2] = d * c.pz[l];
      ch.x[0] = c.x[l]; ch.x[1] = c.y[l]; ch.x[2] = c.z[l];
      ch.tau = tch[e];
      ch.tb = c.t[l];
      ch.id = cid[e];
      ch.w = c.w[l];
      ch.root = c.root[l];
      ch.parent = c.lane[l];
      ch.sp = 2;
      kids.push_back(ch);
      c.px[l] *= od; c.py[l] *= od; c.pz[l] *= od;
      c.tau[l] = tnew[e];
      ++n_emit;
      if (++c.nev[l] >= cfg.max_events) {
        c.gcut[l] = std::numeric_limits<T>::max();
        any_capped = true;
      }
    }
    // 3. particles at the end of the step leave the trip list
    int32_t keep[kChunk];
    for (int l = 0; l < live; ++l) keep[l] = c.t[l] < dt;
    live = compact(c, live, keep);
  }
}

// The photon counterpart: pair rate (eps >= 2), straight line, the photon dies
// at its first event.
template <typename T, bool positions>
void photon_chunk(const Ctx<T>& C, Chunk<T>& c, int n, std::vector<Child<T>>& kids, int64_t& n_pair,
                  uint8_t* dead) {
  const RateRef<T> R = rate_ref(*C.tb, 1);
  const GridRef<T> G = grid_ref(*C.tb, 1);
  const Cfg& cfg = *C.cfg;
  const double dt = C.dt;
  const bool pair = cfg.pair != 0;
#pragma omp simd
  for (int l = 0; l < n; ++l) {
    const T eps = std::sqrt(c.px[l] * c.px[l] + c.py[l] * c.py[l] + c.pz[l] * c.pz[l]);
    const T c2 = chi2_of(c.px[l], c.py[l], c.pz[l], eps, c.ex[l], c.ey[l], c.ez[l], c.bx[l], c.by[l], c.bz[l]);
    const bool on = pair && eps >= T(2) && c2 > T(0);
    c.chi[l] = T(0.5) * std::log(std::max(c2, T(1e-30)));  // ln chi
    c.W[l] = on ? T(kAlpha) / eps : T(0);
  }
#pragma omp simd
  for (int l = 0; l < n; ++l) c.W[l] *= rate_reduced(R, c.chi[l]);
#pragma omp simd
  for (int l = 0; l < n; ++l) {
    const T eps = std::sqrt(c.px[l] * c.px[l] + c.py[l] * c.py[l] + c.pz[l] * c.pz[l]);
    const T W = c.W[l];
    const double rem = dt - c.t[l];
    const double Wr = (double)W * rem;
    const int ev = (W > T(0)) && !(c.tau[l] > Wr);
    double h = ev ? c.tau[l] / (double)W : rem;
    if (h > rem) h = rem;
    c.tau[l] = ev ? c.tau[l] : c.tau[l] - Wr;
    c.t[l] = ev ? c.t[l] + h : dt;
    if (positions && eps > T(0)) {
      const T hh = (T)h / eps;
      c.x[l] += c.px[l] * hh;
      c.y[l] += c.py[l] * hh;
      c.z[l] += c.pz[l] * hh;
    }
    c.ev[l] = ev;
  }
  int ne = 0;
  int32_t idx[kChunk];
  for (int l = 0; l < n; ++l)
    if (c.ev[l]) idx[ne++] = l;
  T xi[kChunk], omx[kChunk];
  double te[kChunk], tp[kChunk];
  uint64_t ide[kChunk], idp[kChunk];
#pragma omp simd
  for (int e = 0; e < ne; ++e) {
    const int l = idx[e];
    const U4 u = philox(C.seed, c.id[l], C.step, 0u);
    const U4 v = philox(C.seed, c.id[l], C.step, 0x80000000u);
    const T z = q_interp(G, c.chi[l], (T)logit_u(u.v[0]));  // logit of the electron's fraction
    xi[e] = T(1) / (T(1) + std::exp(-z));
    omx[e] = T(1) / (T(1) + std::exp(z));
    te[e] = neg_log_u(u.v[2]);
    tp[e] = neg_log_u(u.v[3]);
    ide[e] = (uint64_t)v.v[0] | ((uint64_t)v.v[1] << 32);
    idp[e] = (uint64_t)v.v[2] | ((uint64_t)v.v[3] << 32);
  }
  for (int e = 0; e < ne; ++e) {
    const int l = idx[e];
    const T a = xi[e], b = omx[e];
    for (int k = 0; k < 2; ++k) {
      const T f = k == 0 ? a : b;
      Child<T> ch;
      ch.p[0] = f * c.px[l]; ch.p[1] = f * c.py[l]; ch.p[2] = f * c.pz[l];
      ch.x[0] = c.x[l]; ch.x[1] = c.y[l]; ch.x[2] = c.z[l];
      ch.tau = k == 0 ? te[e] : tp[e];
      ch.tb = c.t[l];
      ch.id = k == 0 ? ide[e] : idp[e];
      ch.w = c.w[l];
      ch.root = c.root[l];
      ch.parent = c.lane[l];
      ch.sp = k;
      kids.push_back(ch);
    }
    c.nev[l] = 1;
    dead[c.lane[l]] = 1;
    ++n_pair;
  }
}

struct Stats {
  int64_t n_emit, n_pair, n_new[3], n_rounds, overflow;
};

// One range [lo, hi) of a species: chunks over OpenMP threads, then the
// children appended in particle order (then event order), as one thread would.
template <typename T>
void run_range(const Ctx<T>& C, Species<T>* app, Stats& st, Species<T>& s, int sp, int64_t lo, int64_t hi,
               bool from_main) {
  if (hi <= lo) return;
  const int64_t nchunks = (hi - lo + kChunk - 1) / kChunk;
  std::vector<std::vector<Child<T>>> out(nchunks);
  std::vector<int64_t> per(nchunks * 3, 0);  // children of each chunk per species, then their first offset
  int64_t n_emit = 0, n_pair = 0;
  bool capped = false;
#pragma omp parallel reduction(+ : n_emit, n_pair) reduction(|| : capped)
  {
    Chunk<T> c;
    std::vector<Child<T>> sorted;
#pragma omp for schedule(dynamic, 4)
    for (int64_t k = 0; k < nchunks; ++k) {
      const int64_t a = lo + k * kChunk;
      const int n = (int)std::min<int64_t>(kChunk, hi - a);
      std::vector<Child<T>>& kids = out[k];
      if (sp < 2) {
        load_chunk(C, s, sp, from_main, a, n, c);
        const T q = sp == 0 ? T(-1) : T(1);
        if (C.cfg->push)
          C.cfg->positions ? lepton_chunk<T, true, true>(C, c, n, q, kids, n_emit, capped)
                           : lepton_chunk<T, true, false>(C, c, n, q, kids, n_emit, capped);
        else
          C.cfg->positions ? lepton_chunk<T, false, true>(C, c, n, q, kids, n_emit, capped)
                           : lepton_chunk<T, false, false>(C, c, n, q, kids, n_emit, capped);
        store_chunk(C, s, a, n, c);
      } else {
        // photons that died in an earlier round leave the chunk before the trip
        load_chunk(C, s, sp, from_main, a, n, c);
        int32_t keep[kChunk];
        for (int l = 0; l < n; ++l) keep[l] = !s.alive || s.alive[a + l];
        const int m = compact(c, n, keep);
        uint8_t dead[kChunk] = {0};
        if (C.cfg->positions)
          photon_chunk<T, true>(C, c, m, kids, n_pair, dead);
        else
          photon_chunk<T, false>(C, c, m, kids, n_pair, dead);
        for (int l = 0; l < m; ++l) {
          const int64_t i = a + c.lane[l];
          if (C.cfg->positions) {
            s.x[i] = c.x[l]; s.y[i] = c.y[l]; s.z[i] = c.z[l];
          }
          s.tau[i] = c.tau[l];
          if (s.nev) s.nev[i] = c.nev[l];
          if (dead[c.lane[l]] && s.alive) s.alive[i] = 0;
        }
      }
      // children of one parent stay in event order, parents in index order
      // (a counting sort over the parent's lane)
      int32_t start[kChunk + 1] = {0};
      for (const Child<T>& ch : kids) ++start[ch.parent + 1];
      for (int l = 0; l < kChunk; ++l) start[l + 1] += start[l];
      sorted.resize(kids.size());
      for (const Child<T>& ch : kids) sorted[start[ch.parent]++] = ch;
      kids.swap(sorted);
      for (const Child<T>& ch : kids) ++per[k * 3 + ch.sp];
    }
  }
  st.n_emit += n_emit;
  st.n_pair += n_pair;
  (void)capped;
  // offsets of each chunk's children in the append stores, then the copy in parallel
  int64_t base[3] = {app[0].count, app[1].count, app[2].count};
  for (int64_t k = 0; k < nchunks; ++k)
    for (int sp2 = 0; sp2 < 3; ++sp2) {
      const int64_t c = per[k * 3 + sp2];
      per[k * 3 + sp2] = base[sp2];
      base[sp2] += c;
    }
  for (int sp2 = 0; sp2 < 3; ++sp2) {
    st.n_new[sp2] += base[sp2] - app[sp2].count;
    if (base[sp2] > app[sp2].capacity) st.overflow = 1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < nchunks; ++k) {
    int64_t at[3] = {per[k * 3], per[k * 3 + 1], per[k * 3 + 2]};
    for (const Child<T>& ch : out[k]) {
      Species<T>& a = app[ch.sp];
      const int64_t i = at[ch.sp]++;
      if (i >= a.capacity) continue;  // overflow: nothing is written past the capacity
      a.px[i] = ch.p[0]; a.py[i] = ch.p[1]; a.pz[i] = ch.p[2];
      if (C.cfg->positions) {
        a.x[i] = ch.x[0]; a.y[i] = ch.x[1]; a.z[i] = ch.x[2];
      }
      a.w[i] = ch.w;
      a.tau[i] = ch.tau;
      a.t_birth[i] = ch.tb;
      a.id[i] = ch.id;
      a.root[i] = ch.root;
      if (a.alive) a.alive[i] = 1;
      if (a.nev) a.nev[i] = 0;
    }
  }
  for (int sp2 = 0; sp2 < 3; ++sp2) app[sp2].count = base[sp2];
}

template <typename T>
int step_impl(const Tables<T>& tb, const Cfg& cfg, Species<T>* main, const Fields<T>* f, Species<T>* app, double dt,
              uint64_t seed, uint32_t step, Stats* st) {
  std::memset(st, 0, sizeof(*st));
  Ctx<T> C{&tb, f, &cfg, dt, seed, step};
  for (int s = 0; s < 3; ++s) app[s].count = 0;
  auto stored = [&](int sp) { return std::min(app[sp].count, app[sp].capacity); };
  run_range(C, app, *st, main[0], 0, 0, main[0].count, true);
  run_range(C, app, *st, main[1], 1, 0, main[1].count, true);
  run_range(C, app, *st, main[2], 2, 0, main[2].count, true);
  int64_t ph_lo = stored(2);
  run_range(C, app, *st, app[2], 2, 0, ph_lo, false);
  int64_t lep_lo = 0, lep_hi = stored(0);
  int64_t rounds = 1;
  while (!st->overflow && lep_hi > lep_lo) {
    run_range(C, app, *st, app[0], 0, lep_lo, lep_hi, false);
    run_range(C, app, *st, app[1], 1, lep_lo, lep_hi, false);
    const int64_t ph_hi = stored(2);
    run_range(C, app, *st, app[2], 2, ph_lo, ph_hi, false);
    ph_lo = ph_hi;
    lep_lo = lep_hi;
    lep_hi = stored(0);
    ++rounds;
  }
  st->n_rounds = rounds;
  return st->overflow ? 2 : 0;
}

}  // namespace

// ------------------------------------------------------------------------------- C interface
extern "C" {

typedef struct {
  int32_t nr;
  double s0, hs;              // rate nodes at ln chi = s0 + i hs
  const double* lnr[2];       // ln of W * energy / alpha (emission, pairs), nr values each
  int32_t rows[2], cols[2];   // inverse-CDF grids (emission, pairs)
  double qs0[2], qhs[2], qx0[2], qhx[2];
  const double* q[2];         // emission: logit(delta) - ln chi; pairs: logit(xi); [rows][cols]
} hs_tables_in;

typedef struct {
  void *px, *py, *pz, *x, *y, *z;
  float* w;
  double* tau;
  uint64_t* id;
  uint8_t* alive;
  int32_t* nev;
  double* t_birth;
  uint32_t* root;
  int64_t count, capacity;
} hs_species;

typedef struct {
  const void *ex, *ey, *ez, *bx, *by, *bz;
  int64_t stride;
} hs_fields;

typedef struct {
  int32_t dtype;  // 0 float, 1 double
  int32_t emission, pair, push, positions;
  double gamma_min;
  int64_t max_events;
  int32_t threads;  // 0: OpenMP's default
} hs_cfg;

typedef struct {
  int64_t n_emit, n_pair, n_new[3], n_rounds, overflow;
} hs_stats;

}  // extern "C"

namespace {

template <typename T>
void* make_tables(const hs_tables_in* in) {
  auto* t = new Tables<T>();
  t->nr = in->nr;
  t->s0 = (T)in->s0;
  t->inv_hr = (T)(1.0 / in->hs);
  for (int p = 0; p < 2; ++p) {
    t->lnr[p].assign(in->lnr[p], in->lnr[p] + in->nr);
    t->rows[p] = in->rows[p];
    t->cols[p] = in->cols[p];
    t->qs0[p] = (T)in->qs0[p];
    t->inv_qhs[p] = (T)(1.0 / in->qhs[p]);
    t->qx0[p] = (T)in->qx0[p];
    t->inv_qhx[p] = (T)(1.0 / in->qhx[p]);
    t->q[p].assign(in->q[p], in->q[p] + (size_t)in->rows[p] * in->cols[p]);
  }
  return t;
}

template <typename T>
Species<T> sp_of(const hs_species& s) {
  return Species<T>{static_cast<T*>(s.px), static_cast<T*>(s.py), static_cast<T*>(s.pz), static_cast<T*>(s.x),
                    static_cast<T*>(s.y), static_cast<T*>(s.z), s.w, s.tau, s.id, s.alive, s.nev, s.t_birth, s.root,
                    s.count, s.capacity};
}

template <typename T>
int step_t(const void* tables, const hs_cfg* cfg, hs_species* main, const hs_fields* f, hs_species* app,
                  double dt, uint64_t seed, uint32_t step, hs_stats* st) {
  Species<T> m[3], a[3];
  Fields<T> F[3];
  for (int s = 0; s < 3; ++s) {
    m[s] = sp_of<T>(main[s]);
    a[s] = sp_of<T>(app[s]);
    F[s] = Fields<T>{static_cast<const T*>(f[s].ex), static_cast<const T*>(f[s].ey), static_cast<const T*>(f[s].ez),
                     static_cast<const T*>(f[s].bx), static_cast<const T*>(f[s].by), static_cast<const T*>(f[s].bz),
                     f[s].stride};
  }
  Cfg c{cfg->emission, cfg->pair, cfg->push, cfg->positions, cfg->gamma_min, cfg->max_events};
  Stats S;
  const int rc = step_impl(*static_cast<const Tables<T>*>(tables), c, m, F, a, dt, seed, step, &S);
  for (int s = 0; s < 3; ++s) app[s].count = a[s].count;
  std::memcpy(st, &S, sizeof(S));
  return rc;
}

}  // namespace

extern "C" {

void* hs_tables_create(const hs_tables_in* in, int32_t dtype) {
  if (!in || in->nr < 4 || !in->lnr[0] || !in->lnr[1]) return nullptr;
  for (int p = 0; p < 2; ++p)
    if (in->rows[p] < 4 || in->cols[p] < 4 || !in->q[p]) return nullptr;
  return dtype == 0 ? make_tables<float>(in) : make_tables<double>(in);
}

void hs_tables_free(void* t, int32_t dtype) {
  if (!t) return;
  if (dtype == 0)
    delete static_cast<Tables<float>*>(t);
  else
    delete static_cast<Tables<double>*>(t);
}

// One global step of the ensemble (Algorithms 1-3); returns 0, 1 (argument
// error) or 2 (an append store overflowed: counts hold the sizes needed).
int hs_step(const void* tables, const hs_cfg* cfg, hs_species main[3], const hs_fields f[3], hs_species app[3],
            double dt, uint64_t seed, uint32_t step, hs_stats* st) {
  if (!tables || !cfg || !main || !f || !app || !st) return 1;
  for (int s = 0; s < 3; ++s) {
    if (app[s].capacity > 0 && (!app[s].t_birth || !app[s].root)) return 1;
    if (s == 2 && ((main[s].count > 0 && !main[s].alive) || (app[s].capacity > 0 && !app[s].alive))) return 1;
    if (cfg->positions && ((main[s].count > 0 && !main[s].x) || (app[s].capacity > 0 && !app[s].x))) return 1;
  }
  if (cfg->threads > 0) omp_set_num_threads(cfg->threads);
  return cfg->dtype == 0 ? step_t<float>(tables, cfg, main, f, app, dt, seed, step, st)
                         : step_t<double>(tables, cfg, main, f, app, dt, seed, step, st);
}

// The tables as the step reads them, one value at a time (for validation):
// W * energy / alpha at chi (proc 0 emission, 1 pairs), and the sampled
// fraction (delta, or the electron's xi) at chi for raw uniforms k.
void hs_eval_rate(const void* tables, int32_t dtype, int32_t proc, const double* chi, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    if (dtype == 0) {
      const RateRef<float> R = rate_ref(*static_cast<const Tables<float>*>(tables), proc);
      out[i] = rate_reduced(R, (float)std::log(chi[i]));
    } else {
      const RateRef<double> R = rate_ref(*static_cast<const Tables<double>*>(tables), proc);
      out[i] = rate_reduced(R, std::log(chi[i]));
    }
  }
}

void hs_sample(const void* tables, int32_t dtype, int32_t proc, const double* chi, const uint32_t* k, int64_t n,
               double* out) {
  for (int64_t i = 0; i < n; ++i) {
    const double s = std::log(chi[i]);
    if (dtype == 0) {
      const GridRef<float> G = grid_ref(*static_cast<const Tables<float>*>(tables), proc);
      const float z = q_interp(G, (float)s, (float)logit_u(k[i])) + (proc == 0 ? (float)s : 0.f);
      out[i] = 1.f / (1.f + std::exp(-z));
    } else {
      const GridRef<double> G = grid_ref(*static_cast<const Tables<double>*>(tables), proc);
      const double z = q_interp(G, s, logit_u(k[i])) + (proc == 0 ? s : 0.0);
      out[i] = 1.0 / (1.0 + std::exp(-z));
    }
  }
}

int32_t hs_max_threads(void) { return omp_get_max_threads(); }
const char* hs_isa(void) { return HS_ISA; }

}  // extern "C"
